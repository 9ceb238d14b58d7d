"""Several right-hand sides in one call (nrhs > 1 in rz_apply, rz_relax, rz_vcycle,
rz_solve).  Multi-vectors are (ndofs, nrhs) tensors, DoF-major with the right-hand
side fastest.  A multi-vector call does per vector the arithmetic of a call on that
vector alone (the H(grad) patch solve reads each factor once for two vectors
but keeps every vector's sums in the same order), so every result must equal the
single-vector call bit for bit; one right-hand side of each solve is also checked
against the oracle's direct solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm

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


def multi(ndofs, seeds, mask=None, dtype=torch.float64):
    m = np.stack([synth.uniform_pm1(s, ndofs) for s in seeds], axis=1)
    if mask is not None:
        m[mask] = 0.0
    return torch.as_tensor(np.ascontiguousarray(m), dtype=dtype, device="cuda:0")


def columns_equal(op, X, Y, dtype=torch.float64):
    """Y[:, r] == op(X[:, r]) bit for bit for every column r."""
    torch.cuda.synchronize()
    for r in range(X.shape[1]):
        y1 = torch.empty(X.shape[0], dtype=dtype, device="cuda:0")
        op(X[:, r].contiguous(), y1)
        torch.cuda.synchronize()
        assert torch.equal(y1, Y[:, r]), f"column {r}: max diff {float((y1 - Y[:, r]).abs().max())}"


PROBLEMS = [
    # (label, kwargs): Cartesian H(grad) with the register patch solve (p = 3, 7),
    # FP64 streaming patch solve (p = 8), trilinear cells, H(curl), H(div)
    ("grad-p3", dict(n=(3, 2, 4), p=3, space="grad")),
    ("grad-p7", dict(n=2, p=7, space="grad")),
    ("grad-p8", dict(n=2, p=8, space="grad")),
    ("quad-p4", dict(n=2, p=4, space="grad", perturb=True)),
    ("curl-p3", dict(n=2, p=3, space="curl")),
    ("div-p2", dict(n=2, p=2, space="div")),
]


def make(rz, ctx, kw, precision=0):
    n, p, space = kw["n"], kw["p"], kw["space"]
    nn = (n, n, n) if np.isscalar(n) else n
    nc = nn[0] * nn[1] * nn[2]
    al = synth.cell_coefficients(nc, 1, 0.1, 10.0)
    be = synth.cell_coefficients(nc, 2, 0.1, 10.0)
    if kw.get("perturb"):
        verts = synth.perturbed_vertices(n, 5, 0.1)
        return rz.Problem(ctx, n, p, al, be, space=space, vertices=verts, precision=precision)
    return rz.Problem(ctx, n, p, al, be, space=space, precision=precision)


@pytest.mark.parametrize("label,kw", PROBLEMS, ids=[l for l, _ in PROBLEMS])
def test_apply_relax_vcycle_multi(rz, ctx, label, kw):
    print(f"multi-RHS apply/relax/vcycle {label}", flush=True)
    pb = make(rz, ctx, kw)
    try:
        for nrhs in (3, 4, 6):
            X = multi(pb.ndofs, range(10, 10 + nrhs))
            Y = torch.empty_like(X)
            pb.apply(X, Y)
            columns_equal(pb.apply, X, Y)
            pb.relax(X, Y)
            columns_equal(pb.relax, X, Y)
            pb.vcycle(X, Y)
            columns_equal(pb.vcycle, X, Y)
        X32 = multi(pb.ndofs, range(20, 25), dtype=torch.float32)
        Y32 = torch.empty_like(X32)
        pb.apply(X32, Y32, rz.F32)
        columns_equal(lambda a, b: pb.apply(a, b, rz.F32), X32, Y32, torch.float32)
        pb.relax(X32, Y32, rz.F32)
        columns_equal(lambda a, b: pb.relax(a, b, rz.F32), X32, Y32, torch.float32)
    finally:
        pb.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("label,kw", [PROBLEMS[1], PROBLEMS[0], PROBLEMS[4]], ids=["grad-p7", "grad-p3", "curl-p3"])
def test_solve_multi_equals_single(rz, ctx, label, kw, precision):
    print(f"multi-RHS solve {label} precision={precision}", flush=True)
    pb = make(rz, ctx, kw, precision)
    try:
        nrhs = 4
        B = multi(pb.ndofs, range(30, 30 + nrhs))
        B[:, 2] *= 1e-3  # right-hand sides of different size converge at their own pace
        X = torch.empty_like(B)
        infos = pb.solve(B, X)
        assert len(infos) == nrhs
        torch.cuda.synchronize()
        for r in range(nrhs):
            x1 = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
            info = pb.solve(B[:, r].contiguous(), x1)
            torch.cuda.synchronize()
            assert info.iters == infos[r].iters
            assert info.iters_natural == infos[r].iters_natural
            assert infos[r].rel_res <= 1e-8
            assert torch.equal(x1, X[:, r])
        # one right-hand side against the oracle's direct solve
        n = kw["n"]
        nn = (n, n, n) if np.isscalar(n) else n
        if kw["space"] == "grad":
            nc = nn[0] * nn[1] * nn[2]
            lat = Lattice(Mesh(*nn), "grad", kw["p"])
            A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, synth.cell_coefficients(nc, 1, 0.1, 10.0),
                                                              synth.cell_coefficients(nc, 2, 0.1, 10.0)))
            b0 = np.where(lat.dirichlet_mask(), 0.0, B[:, 1].cpu().numpy())
            xs0 = spla.spsolve(A.tocsc(), b0)
            x0 = X[:, 1].cpu().numpy()
            assert np.linalg.norm(x0 - xs0) <= 1e-6 * np.linalg.norm(xs0)
    finally:
        pb.close()


def test_solve_multi_zero_column(rz, ctx):
    """A zero right-hand side among others: x = 0 after no iteration, the others as
    alone."""
    pb = make(rz, ctx, PROBLEMS[0][1])
    try:
        B = multi(pb.ndofs, [40, 41, 42])
        B[:, 1] = 0.0
        X = torch.full_like(B, 7.0)
        infos = pb.solve(B, X)
        torch.cuda.synchronize()
        assert infos[1].iters == 0 and infos[1].status == 0
        assert float(X[:, 1].abs().max()) == 0.0
        for r in (0, 2):
            x1 = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
            pb.solve(B[:, r].contiguous(), x1)
            torch.cuda.synchronize()
            assert torch.equal(x1, X[:, r])
    finally:
        pb.close()


def test_solve_multi_not_converged(rz, ctx):
    """maxit = 1: every right-hand side reports RZ_ERR_NOT_CONVERGED and the call
    raises it."""
    pb = rz.Problem(ctx, 3, 3, 1.0, 1.0, maxit=1)
    try:
        B = multi(pb.ndofs, [50, 51])
        X = torch.empty_like(B)
        infos = pb.solve(B, X, check=False)
        assert [i.status for i in infos] == [-4, -4]
        assert [i.iters for i in infos] == [1, 1]
        with pytest.raises(rz.RzError):
            pb.solve(B, X)
    finally:
        pb.close()
