"""GPU parity of the trilinear-cell / sampled-coefficient path against the oracle,
through the C ABI: quadrature apply (Gauss-Lobatto, ceil(3(p+1)/2) points per axis),
relaxation with cell-averaged separable weights, the p=1 coarse solve integrated
with 3 points per axis, and PCG.  Tolerances as for the Cartesian path (FP64
1e-12, FP32 apply 1e-5)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, auxop, matfree, schwarz, pmg
from oracle.quadrature import averaged_coefficients, sample_function, default_points

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
    """Relative error, the larger of the 2-norm one and the per-entry one
    (max |a - b| / max |b|), so that one wrong entry cannot hide in the norm."""
    nb = max(np.linalg.norm(b), 1e-300)
    mb = max(np.abs(b).max(initial=0.0), 1e-300)
    return max(np.linalg.norm(a - b) / nb, np.abs(a - b).max(initial=0.0) / mb)


def T(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


class Ref:
    def __init__(self, n, p, vertices, seed=1):
        self.m = Mesh(*n, vertices=vertices)
        self.lat = Lattice(self.m, "grad", p)
        self.latc = Lattice(self.m, "grad", 1)
        self.a = sample_function(self.m, alpha_fn)
        # beta: positive samples varying per cell
        self.b = np.repeat(synth.cell_coefficients(self.m.ncells, seed + 1, 0.5, 2.0)[:, None], 27, 1)
        self.q = default_points(p)
        self.mask = self.lat.dirichlet_mask()

    def relax(self):
        co = averaged_coefficients(self.m, self.a, self.b, self.q)
        return schwarz.SCRelaxGrad(self.lat, auxop.separable_operator(self.lat, co))

    def operator(self):
        return asm.with_dirichlet(self.lat, asm.quadrature_operator(self.lat, self.a, self.b, self.q, kind="gll"))

    def coarse(self):
        A0 = asm.with_dirichlet(self.latc, asm.quadrature_operator(self.latc, self.a, self.b, default_points(1),
                                                                  kind="gll"))
        return pmg.CoarseSolver(self.latc, A0)


APPLY_CASES = [((3, 2, 2), 1), ((3, 2, 4), 3), ((2, 2, 2), 4), ((3, 3, 2), 7), ((2, 2, 2), 8), ((2, 2, 2), 9)]


@pytest.mark.parametrize("n,p", APPLY_CASES)
def test_quad_apply_parity(rz, ctx, n, p):
    ref = Ref(n, p, perturbed(n))
    pb = rz.Problem(ctx, n, p, ref.a, ref.b, vertices=ref.m.vertices, omega=0.3)
    x = synth.uniform_pm1(7, pb.ndofs)
    y_ref = matfree.apply(ref.lat, x, ref.a, ref.b, ref.q, kind="gll")
    y = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
    pb.apply(T(x), y)
    assert rel(H(y), y_ref) < 1e-12
    y32 = torch.empty(pb.ndofs, dtype=torch.float32, device="cuda:0")
    pb.apply(T(x, torch.float32), y32, rz.F32)
    assert rel(H(y32), y_ref) < 1e-5


def test_quad_apply_on_boxes_equals_kronecker_path(rz, ctx):
    # samples of cellwise constants on a Cartesian mesh: the quadrature path must
    # reproduce the exact Kronecker operator
    n, p = (3, 2, 2), 5
    m = Mesh(*n)
    al = synth.cell_coefficients(m.ncells, 1)
    be = synth.cell_coefficients(m.ncells, 2)
    pq = rz.Problem(ctx, n, p, np.repeat(al[:, None], 27, 1), np.repeat(be[:, None], 27, 1), omega=0.3)
    pk = rz.Problem(ctx, n, p, al, be, omega=0.3)
    x = T(synth.uniform_pm1(8, pq.ndofs))
    yq = torch.empty_like(x)
    yk = torch.empty_like(x)
    pq.apply(x, yq)
    pk.apply(x, yk)
    assert rel(H(yq), H(yk)) < 1e-12


@pytest.mark.parametrize("n,p", [((3, 2, 3), 3), ((2, 2, 2), 8)])
def test_quad_relax_parity(rz, ctx, n, p):
    ref = Ref(n, p, perturbed(n))
    pb = rz.Problem(ctx, n, p, ref.a, ref.b, vertices=ref.m.vertices, omega=0.3)
    assert np.allclose(pb.aux_coefficients(), averaged_coefficients(ref.m, ref.a, ref.b, ref.q), rtol=1e-13)
    r = np.where(ref.mask, 0.0, synth.uniform_pm1(11, ref.lat.ndofs))
    z_ref = ref.relax().apply(r)
    z = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
    pb.relax(T(r), z)
    assert rel(H(z), z_ref) < 1e-12


def test_quad_coarse_parity(rz, ctx):
    n = (4, 3, 3)
    ref = Ref(n, 2, perturbed(n))
    pb = rz.Problem(ctx, n, 2, ref.a, ref.b, vertices=ref.m.vertices, omega=0.3)
    rc = np.where(ref.latc.dirichlet_mask(), 0.0, synth.uniform_pm1(31, ref.latc.ndofs))
    xc = torch.empty(pb.ncoarse, dtype=torch.float64, device="cuda:0")
    pb.coarse_solve(T(rc), xc)
    assert rel(H(xc), ref.coarse().solve(rc)) < 1e-12


def test_quad_hmg_coarse_parity(rz, ctx):
    """The h-multigrid coarse solver (rz_opts.coarse = RZ_COARSE_HMG) on trilinear cells
    with sampled coefficients: level 0 is the quadrature Q_1 operator, the hierarchy
    and one V(1,1) cycle equal the oracle's HMGCoarse on the same operator to 1e-12."""
    n = (16, 8, 8)
    ref = Ref(n, 2, perturbed(n))
    pb = rz.Problem(ctx, n, 2, ref.a, ref.b, vertices=ref.m.vertices, omega=0.3, coarse=rz.COARSE_HMG)
    try:
        A0 = asm.with_dirichlet(ref.latc, asm.quadrature_operator(ref.latc, ref.a, ref.b, default_points(1),
                                                                 kind="gll"))
        hm = pmg.HMGCoarse(ref.latc, A0, min_free=512)
        assert pb.hmg_levels() == [a.shape[0] for a in hm.A] == [735, 63]
        rc = np.where(ref.latc.dirichlet_mask(), 0.0, synth.uniform_pm1(31, ref.latc.ndofs))
        xc = torch.empty(pb.ncoarse, dtype=torch.float64, device="cuda:0")
        pb.coarse_solve(T(rc), xc)
        assert rel(H(xc), hm.solve(rc)) < 1e-12
    finally:
        pb.close()


@pytest.mark.parametrize("n,p,prec", [((3, 3, 3), 4, 0), ((3, 3, 3), 4, 1), ((3, 2, 2), 5, 0)])
def test_quad_solve_parity(rz, ctx, n, p, prec):
    ref = Ref(n, p, perturbed(n))
    A = ref.operator()
    R = ref.relax()
    mask = ref.mask
    v0 = np.where(mask, 0.0, synth.uniform_pm1(99, ref.lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    om = pmg.omega_from_lambda(lam)
    pb = rz.Problem(ctx, n, p, ref.a, ref.b, vertices=ref.m.vertices, precision=prec)
    assert abs(pb.omega() - om) < 1e-6 * om
    Pr = pmg.prolongation(ref.lat, ref.latc)
    b = np.where(mask, 0.0, synth.rhs_values(ref.lat.ndofs, 0))
    x_ref, it_ref, _ = pmg.pcg(A, b, pmg.VCycle(ref.lat, A, R, Pr, ref.coarse(), om))
    x = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
    info = pb.solve(T(b), x)
    xg = H(x)
    xs = spla.spsolve(A.tocsc(), b)
    assert info.rel_res <= 1e-8
    assert np.linalg.norm(b - A @ xg) <= 1e-8 * np.linalg.norm(b)
    eA = np.sqrt((xg - xs) @ (A @ (xg - xs)) / (xs @ (A @ xs)))
    assert eA < 1e-7
    assert abs(info.iters - it_ref) <= (1 if prec == 0 else 2)
