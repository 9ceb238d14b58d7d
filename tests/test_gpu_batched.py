"""Batched solves (rz_solve_batched): problems of uneven size and degree on several
contexts (streams) solved concurrently, several right-hand sides each (multi-vectors
of shape (ndofs, nrhs), the right-hand side fastest).  Every batched result must
equal the single rz_solve of the same problem and right-hand side bit for bit (the
kernels are deterministic, and a multi-vector solve does the arithmetic of separate
solves), reach the tolerance, and the first problem is checked against the oracle's
direct solve."""
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
