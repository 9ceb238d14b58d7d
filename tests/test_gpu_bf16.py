"""BF16 operator apply (rz_apply with RZ_BF16) against the FP64 oracle.

The input x is drawn, rounded to BF16, and the oracle applies the FP64 operator to
that BF16 value exactly, so every difference comes from the BF16 arithmetic of the
library.  Unit roundoff of BF16 (8 significant bits): u = 2^-8.

  * Trilinear cells (matrix-core contractions): the tables B_q, D_q are rounded to
    BF16 (one rounding each), and the results of the x-, y- and z-contractions, the
    pointwise fluxes, and the transposed z- and y-contractions are rounded to BF16
    before the next product (five more roundings), accumulation in FP32, the output
    rounded once.  Each rounding perturbs the quantity it rounds by at most u
    relatively (about u/sqrt(3) RMS); through the contractions that gives an error of
    order sqrt(7) u/sqrt(3) ~ 6e-3 of the magnitudes summed into y, and the
    stiffness terms cancel to up to a few times less than those magnitudes: the test
    accepts 2e-2 relative (2-norm and per entry against max |y|; measured 3.4e-3 to
    5.7e-3 and 5.2e-3 to 8.2e-3 for p = 3, 4, 8, 9), and asserts that the error is
    also above the FP32 level (the BF16 path really ran).
  * Cartesian cells (FP32 line operators on BF16 loads and stores): only the output
    is rounded: per entry |y - y_ref| <= u |y_ref| + 1e-5 max |y_ref| (FP32 sums).
"""
import numpy as np
import pytest

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, matfree
from oracle.quadrature import sample_function, default_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U_BF16 = 2.0 ** -8


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


def bf16_input(ndofs, seed):
    """(device BF16 tensor, its exact FP64 value)."""
    xb = torch.as_tensor(synth.uniform_pm1(seed, ndofs), dtype=torch.float64).to(torch.bfloat16)
    return xb.to("cuda:0"), xb.to(torch.float64).numpy()


def errors(y, ref):
    d = y - ref
    return np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max()


@pytest.mark.parametrize("n,p", [((3, 2, 2), 1), ((2, 2, 3), 3), ((2, 2, 2), 4), ((2, 2, 2), 8), ((2, 2, 2), 9)])
def test_bf16_matrix_core_apply(rz, ctx, n, p):
    print(f"BF16 matrix-core apply n={n} p={p}", flush=True)
    m = Mesh(*n, vertices=perturbed(n))
    a = sample_function(m, alpha_fn)
    b = np.repeat(synth.cell_coefficients(m.ncells, 2, 0.5, 2.0)[:, None], 27, 1)
    pb = rz.Problem(ctx, n, p, a, b, vertices=m.vertices, omega=0.3)
    try:
        lat = Lattice(m, "grad", p)
        x, xr = bf16_input(pb.ndofs, 7)
        y_ref = matfree.apply(lat, xr, a, b, default_points(p), kind="gll")
        y = torch.empty(pb.ndofs, dtype=torch.bfloat16, device="cuda:0")
        pb.apply(x, y, rz.BF16)
        torch.cuda.synchronize()
        e2, emax = errors(y.to(torch.float64).cpu().numpy(), y_ref)
        print(f"  relative error: 2-norm {e2:.3e}, per entry {emax:.3e}", flush=True)
        assert e2 < 2e-2 and emax < 2e-2
        assert e2 > 1e-5  # BF16 arithmetic, not an FP32 or FP64 path
    finally:
        pb.close()


@pytest.mark.parametrize("n,p", [((3, 2, 4), 3), ((2, 3, 2), 7)])
def test_bf16_cartesian_apply(rz, ctx, n, p):
    print(f"BF16 Cartesian apply n={n} p={p}", flush=True)
    m = Mesh(*n)
    al = synth.cell_coefficients(m.ncells, 1)
    be = synth.cell_coefficients(m.ncells, 2)
    pb = rz.Problem(ctx, n, p, al, be, omega=0.3)
    try:
        lat = Lattice(m, "grad", p)
        x, xr = bf16_input(pb.ndofs, 9)
        y_ref = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be)) @ xr
        y = torch.empty(pb.ndofs, dtype=torch.bfloat16, device="cuda:0")
        pb.apply(x, y, rz.BF16)
        torch.cuda.synchronize()
        yh = y.to(torch.float64).cpu().numpy()
        bound = U_BF16 * np.abs(y_ref) + 1e-5 * np.abs(y_ref).max()
        assert np.all(np.abs(yh - y_ref) <= bound)
    finally:
        pb.close()


def test_bf16_multi_vector_equals_single(rz, ctx):
    n, p = (2, 2, 2), 8
    m = Mesh(*n, vertices=perturbed(n))
    a = sample_function(m, alpha_fn)
    pb = rz.Problem(ctx, n, p, a, 1.0, vertices=m.vertices, omega=0.3)
    try:
        X = torch.stack([bf16_input(pb.ndofs, s)[0] for s in (3, 4, 5)], dim=1).contiguous()
        Y = torch.empty_like(X)
        pb.apply(X, Y, rz.BF16)
        torch.cuda.synchronize()
        for r in range(3):
            y1 = torch.empty(pb.ndofs, dtype=torch.bfloat16, device="cuda:0")
            pb.apply(X[:, r].contiguous(), y1, rz.BF16)
            torch.cuda.synchronize()
            assert torch.equal(y1, Y[:, r])
    finally:
        pb.close()


def test_bf16_rejected_for_vector_spaces(rz, ctx):
    pb = rz.Problem(ctx, 2, 2, 1.0, 1.0, space="curl", omega=0.3)
    try:
        x = torch.zeros(pb.ndofs, dtype=torch.bfloat16, device="cuda:0")
        y = torch.empty_like(x)
        with pytest.raises(rz.RzError):
            pb.apply(x, y, rz.BF16)
    finally:
        pb.close()
