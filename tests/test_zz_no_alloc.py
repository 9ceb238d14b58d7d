"""rz_apply_noalloc (the apply with the library's static workspace, no allocation in
the call) against rz_apply, through the C ABI: identical kernels, so the outputs
must agree to FP64 1e-12 / FP32 1e-6 relative and per entry (they are in fact
bit-identical).  Two calls in a row on one GPU, the second on a smaller problem
(the static array keeps the first call's contents), on each apply path (Cartesian
H(grad), quadrature H(grad), H(curl), H(div)); a problem whose workspace exceeds
the static array is rejected with RZ_ERR_ARG."""
import numpy as np
import pytest

import synth

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


def _perturbed(n, seed):
    v = synth.perturbed_vertices(n, seed)
    return v


def _problem(rz, ctx, kind, n, p):
    nc = n ** 3
    al = synth.cell_coefficients(nc, 1)
    be = synth.cell_coefficients(nc, 2)
    if kind == "grad":
        return rz.Problem(ctx, n, p, al, be, omega=0.3)
    if kind == "quad":
        v = _perturbed(n, 3)
        return rz.Problem(ctx, n, p, synth.c5_coefficient_samples(v, n), 1.0, vertices=v, omega=0.3)
    return rz.Problem(ctx, n, p, al, be, space=kind)


def _check(rz, pb, seed):
    for dt, code, tol in ((torch.float64, rz.F64, 1e-12), (torch.float32, rz.F32, 1e-6)):
        x = torch.as_tensor(synth.uniform_pm1(seed, pb.ndofs), dtype=dt, device="cuda:0")
        y_ref = torch.empty_like(x)
        y_na = torch.full_like(x, float("nan"))
        pb.apply(x, y_ref, code)
        pb.apply_noalloc(x, y_na, code)
        torch.cuda.synchronize()
        a, b = y_na.double().cpu().numpy(), y_ref.double().cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b)
        assert np.max(np.abs(a - b)) <= tol * np.max(np.abs(b))


@pytest.mark.parametrize("kind,big,small", [("grad", (12, 7), (3, 4)), ("quad", (5, 8), (2, 3)),
                                            ("curl", (6, 6), (2, 3)), ("div", (5, 5), (3, 2))])
def test_noalloc_matches_apply_twice(rz, ctx, kind, big, small):
    print(f"noalloc {kind} big={big} small={small}", flush=True)
    p1 = _problem(rz, ctx, kind, *big)
    p2 = _problem(rz, ctx, kind, *small)
    _check(rz, p1, 21)
    _check(rz, p2, 22)   # second call, smaller input: stale contents must not leak in
    p1.close()
    p2.close()


def test_noalloc_rejects_oversized_workspace(rz, ctx):
    # NCE_9 on 12^3 cells: 3 contributions x 3,849,444 DoFs x 8 B = 92.4 MB > 64 MiB
    pb = rz.Problem(ctx, 12, 9, 1.0, 1.0, space="curl")
    x = torch.zeros(pb.ndofs, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    with pytest.raises(rz.RzError) as ei:
        pb.apply_noalloc(x, y)
    assert ei.value.code == -1
    # FP32 needs half of it and runs
    x32, y32 = x.float(), y.float()
    pb.apply_noalloc(x32, y32, rz.F32)
    torch.cuda.synchronize()
    pb.close()
