"""GPU parity of the H(grad) relaxation with the paper's auxiliary operator
(RZ_AUX_PAPER_DIAG: eq. sum-factorization_approx, the weighted mass matrices
replaced by their diagonals in the broken bases) on trilinear cells with sampled
coefficients, against the oracle (auxop.paper_operator with the same samples and the
GLL rule of the apply, relaxed by schwarz.SCRelaxGrad), through the C ABI.

Tolerances as for the separable path: broken diagonals and the FP64 relaxation
1e-12 relative (2-norm and per entry), FP32 relaxation 1e-4, V-cycle 1e-11, solve
iteration count within one of the oracle's PCG, true residual <= 1e-8 and A-norm
error against a direct solve below 1e-7."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, auxop, schwarz, pmg
from oracle.tables1d import Element1D
from oracle.quadrature import sample_function, default_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14284_amd import rz as mod
    return mod


@pytest.fixture(scope="module")
def ctx(rz):
    return rz.Context(0, torch.cuda.current_stream())


def alpha_fn(X):
    return np.exp(0.5 * np.sin(2 * np.pi * X[:, 0]) * np.sin(2 * np.pi * X[:, 1]) * np.sin(2 * np.pi * X[:, 2]))


def perturbed(n, seed=3):
    nx, ny, nz = n
    m = Mesh(nx, ny, nz)
    v = m.vertices.copy()
    u = synth.uniform_pm1(seed, v.size).reshape(v.shape)
    k = np.arange(v.shape[0])
    ix, iy, iz = k % (nx + 1), (k // (nx + 1)) % (ny + 1), k // ((nx + 1) * (ny + 1))
    inner = (ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)
    v[inner] += 0.15 * np.array([1.0 / nx, 1.0 / ny, 1.0 / nz]) * u[inner]
    return v


def rel(a, b):
    nb = max(np.linalg.norm(b), 1e-300)
    mb = max(np.abs(b).max(initial=0.0), 1e-300)
    return max(np.linalg.norm(a - b) / nb, np.abs(a - b).max(initial=0.0) / mb)


def T(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


class Ref:
    def __init__(self, n, p):
        self.m = Mesh(*n, vertices=perturbed(n))
        self.p = p
        self.lat = Lattice(self.m, "grad", p)
        self.latc = Lattice(self.m, "grad", 1)
        self.a = sample_function(self.m, alpha_fn)
        self.b = np.repeat(synth.cell_coefficients(self.m.ncells, 4, 0.5, 2.0)[:, None], 27, 1)
        self.q = default_points(p)
        self.mask = self.lat.dirichlet_mask()
        self.P = asm.with_dirichlet(self.lat, auxop.paper_operator(self.lat, self.a, self.b, q=self.q, kind="gll"))
        self.R = schwarz.SCRelaxGrad(self.lat, self.P)

    def operator(self):
        return asm.with_dirichlet(self.lat, asm.quadrature_operator(self.lat, self.a, self.b, self.q, kind="gll"))

    def coarse(self):
        A0 = asm.with_dirichlet(self.latc, asm.quadrature_operator(self.latc, self.a, self.b, default_points(1),
                                                                  kind="gll"))
        return pmg.CoarseSolver(self.latc, A0)


def problem(rz, ctx, ref, **kw):
    return rz.Problem(ctx, ref.m.n, ref.p, ref.a, ref.b, vertices=ref.m.vertices, aux=rz.AUX_PAPER_DIAG, **kw)


CASES = [((2, 2, 2), 3), ((3, 2, 2), 4), ((2, 2, 2), 7), ((2, 2, 2), 8)]


@pytest.mark.parametrize("n,p", CASES)
def test_paper_diagonals_and_relax(rz, ctx, n, p):
    print(f"paper auxiliary n={n} p={p}", flush=True)
    ref = Ref(n, p)
    pb = problem(rz, ctx, ref, omega=0.3)
    try:
        el = Element1D(p)
        cv = ref.m.cell_vertices()
        for c in (0, ref.m.ncells - 1):
            dm, da = pb.paper_diagonals(c)
            dm_r, da_r = auxop.paper_diagonals_grad(el, cv[c], ref.a[c], ref.b[c], ref.q, kind="gll")
            assert rel(dm, dm_r) < 1e-12
            for m in range(3):
                assert rel(da[m], da_r[m]) < 1e-12
        r = np.where(ref.mask, 0.0, synth.uniform_pm1(11, ref.lat.ndofs))
        z_ref = ref.R.apply(r)
        z = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
        pb.relax(T(r), z)
        assert rel(H(z), z_ref) < 1e-12
        z32 = torch.empty(pb.ndofs, dtype=torch.float32, device="cuda:0")
        pb.relax(T(r, torch.float32), z32, rz.F32)
        assert rel(H(z32), z_ref) < 1e-4
    finally:
        pb.close()


@pytest.mark.parametrize("n,p,prec", [((3, 3, 3), 4, 0), ((3, 3, 3), 4, 1), ((3, 2, 2), 5, 0)])
def test_paper_aux_solve(rz, ctx, n, p, prec):
    print(f"paper auxiliary solve n={n} p={p} prec={prec}", flush=True)
    ref = Ref(n, p)
    A = ref.operator()
    R = ref.R
    mask = ref.mask
    v0 = np.where(mask, 0.0, synth.uniform_pm1(99, ref.lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    om = pmg.omega_from_lambda(lam)
    pb = problem(rz, ctx, ref, precision=prec)
    try:
        assert abs(pb.omega() - om) < 1e-6 * om
        Pr = pmg.prolongation(ref.lat, ref.latc)
        b = np.where(mask, 0.0, synth.rhs_values(ref.lat.ndofs, 0))
        _, it_ref, _ = pmg.pcg(A, b, pmg.VCycle(ref.lat, A, R, Pr, ref.coarse(), om))
        x = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
        info = pb.solve(T(b), x)
        xg = H(x)
        xs = spla.spsolve(A.tocsc(), b)
        assert info.rel_res <= 1e-8
        assert np.linalg.norm(b - A @ xg) <= 1e-8 * np.linalg.norm(b)
        eA = np.sqrt((xg - xs) @ (A @ (xg - xs)) / (xs @ (A @ xs)))
        assert eA < 1e-7
        print(f"  iterations: library {info.iters}, oracle {it_ref}", flush=True)
        assert abs(info.iters - it_ref) <= (1 if prec == 0 else 2)
    finally:
        pb.close()


def test_paper_aux_multi_vector_and_set_aux(rz, ctx):
    ref = Ref((2, 2, 2), 4)
    pb = problem(rz, ctx, ref, omega=0.3)
    try:
        X = torch.stack([T(np.where(ref.mask, 0.0, synth.uniform_pm1(s, pb.ndofs))) for s in (1, 2, 3)], 1)
        X = X.contiguous()
        Z = torch.empty_like(X)
        pb.relax(X, Z)
        torch.cuda.synchronize()
        for r in range(3):
            z1 = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
            pb.relax(X[:, r].contiguous(), z1)
            torch.cuda.synchronize()
            assert torch.equal(z1, Z[:, r])
        with pytest.raises(rz.RzError):
            pb.set_aux(np.ones((pb.ncells, 6)))
    finally:
        pb.close()
