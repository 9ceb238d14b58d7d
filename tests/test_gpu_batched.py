"""Batched solves (rz_solve_batched): problems of uneven size and degree on several
contexts (streams) solved concurrently, several right-hand sides each (multi-vectors
of shape (ndofs, nrhs), the right-hand side fastest).  Every batched result must
equal the single rz_solve of the same problem and right-hand side bit for bit (the
kernels are deterministic, and a multi-vector solve does the arithmetic of separate
solves) and reach the tolerance.  A batch with members of all three spaces is checked
member by member against the oracle's direct solves, and a member stopped by its
iteration cap reports its status without stopping the others."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPECS = [(3, 4), (4, 3), (2, 7), (5, 2), (3, 5), (4, 6)]


def test_batched_equals_single_solves():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14284_amd import rz
    streams = [torch.cuda.Stream() for _ in range(3)]
    ctxs = [rz.Context(0, s) for s in streams]
    probs, bs, xs = [], [], []
    nrhs = 2
    for i, (n, p) in enumerate(SPECS):
        pb = rz.Problem(ctxs[i % 3], n, p, 1.0, 1.0)
        probs.append(pb)
        b = np.stack([synth.rhs_values(pb.ndofs, 4 * i + r) for r in range(nrhs)], axis=1)
        bs.append(torch.as_tensor(np.ascontiguousarray(b), device="cuda:0"))
        xs.append(torch.zeros((pb.ndofs, nrhs), dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    infos = rz.solve_batched(probs, bs, xs)
    torch.cuda.synchronize()
    for i, pb in enumerate(probs):
        for r in range(nrhs):
            assert infos[i][r].rel_res <= 1e-8
            x1 = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
            with torch.cuda.stream(streams[i % 3]):
                info = pb.solve(bs[i][:, r].contiguous(), x1)
            torch.cuda.synchronize()
            assert info.iters == infos[i][r].iters
            assert torch.equal(x1, xs[i][:, r])
    n, p = SPECS[0]
    lat = Lattice(Mesh(n, n, n), "grad", p)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.0, 1.0))
    b0 = np.where(lat.dirichlet_mask(), 0.0, bs[0][:, 0].cpu().numpy())
    xs0 = spla.spsolve(A.tocsc(), b0)
    x0 = xs[0][:, 0].cpu().numpy()
    assert np.linalg.norm(x0 - xs0) < 1e-6 * np.linalg.norm(xs0)


@pytest.mark.parametrize("graph", [0, 1])
def test_batched_reports_a_failing_member(graph):
    """A member stopped by maxit = 1 reports RZ_ERR_NOT_CONVERGED in its infos, the
    other members still converge, and the call returns that status (check=True
    raises it), with and without captured iterations."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14284_amd import rz
    streams = [torch.cuda.Stream() for _ in range(2)]
    ctxs = [rz.Context(0, s) for s in streams]
    probs = [rz.Problem(ctxs[0], 3, 4, 1.0, 1.0, graph=graph),
             rz.Problem(ctxs[1], 3, 3, 1.0, 1.0, maxit=1, graph=graph),
             rz.Problem(ctxs[0], 2, 3, 1.0, 1.0, space="curl", graph=graph)]
    try:
        bs = [torch.as_tensor(np.ascontiguousarray(np.stack([synth.rhs_values(pb.ndofs, 60 + 2 * i + r)
                                                             for r in range(2)], axis=1)), device="cuda:0")
              for i, pb in enumerate(probs)]
        xs = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        infos = rz.solve_batched(probs, bs, xs, check=False)
        torch.cuda.synchronize()
        assert [i.status for i in infos[1]] == [-4, -4]
        assert [i.iters for i in infos[1]] == [1, 1]
        for k in (0, 2):
            assert all(i.status == 0 and i.rel_res <= 1e-8 for i in infos[k])
        with pytest.raises(rz.RzError) as ei:
            rz.solve_batched(probs, bs, xs)
        assert ei.value.code == -4
    finally:
        for pb in probs:
            pb.close()
        for c in ctxs:
            c.close()


MIXED = [("grad", 3, 4), ("curl", 2, 3), ("div", 2, 4), ("grad", 2, 6), ("curl", 3, 2), ("div", 3, 2)]


def test_batched_all_spaces_against_oracle():
    """Members of all three spaces in one batched call, two right-hand sides each:
    every member and right-hand side against the oracle's direct solve of the
    assembled operator (relative 2-norm error below 1e-6, A-norm below 1e-7)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14284_amd import rz
    streams = [torch.cuda.Stream() for _ in range(2)]
    ctxs = [rz.Context(0, s) for s in streams]
    probs, bs = [], []
    try:
        for i, (space, n, p) in enumerate(MIXED):
            pb = rz.Problem(ctxs[i % 2], n, p, 1.0, 1.0, space=space)
            probs.append(pb)
            b = np.stack([synth.rhs_values(pb.ndofs, 80 + 2 * i + r) for r in range(2)], axis=1)
            bs.append(torch.as_tensor(np.ascontiguousarray(b), device="cuda:0"))
        xs = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        infos = rz.solve_batched(probs, bs, xs)
        torch.cuda.synchronize()
        for i, (space, n, p) in enumerate(MIXED):
            lat = Lattice(Mesh(n, n, n), space, p)
            A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.0, 1.0)).tocsc()
            mask = lat.dirichlet_mask()
            for r in range(2):
                assert infos[i][r].rel_res <= 1e-8
                b = np.where(mask, 0.0, bs[i][:, r].cpu().numpy())
                xr = spla.spsolve(A, b)
                x = xs[i][:, r].cpu().numpy()
                e = x - xr
                assert np.linalg.norm(e) < 1e-6 * np.linalg.norm(xr), (space, n, p, r)
                assert np.sqrt(e @ (A @ e) / (xr @ (A @ xr))) < 1e-7, (space, n, p, r)
    finally:
        for pb in probs:
            pb.close()
        for c in ctxs:
            c.close()
