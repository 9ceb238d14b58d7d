"""Solves with captured HIP graphs (rz_opts.graph = 1) against the same solves with
launches one by one (graph = 0), through the C ABI.

The graphs replay the same kernels with the same arguments in the same order, so the
solutions and iteration counts must be identical bit for bit: H(grad) in the FP64 and
mixed protocols (the cooperative Q_1 coarse solve runs between graph segments),
H(curl) and H(div) (one graph per iteration), one and several right-hand sides,
repeated solves (replay of the captured graphs), a new x vector (new capture), a
larger right-hand-side count after a smaller one (the multi-vector buffers are
replaced, the graphs captured again), and the batched driver.  The solves reach a
true relative residual of 1e-8."""
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
    c = rz.Context(0, torch.cuda.current_stream())
    yield c


def rhs(pb, seeds):
    cols = [synth.rhs_values(pb.ndofs, s) for s in seeds]
    a = np.stack(cols, axis=1) if len(cols) > 1 else cols[0]
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


CASES = [("grad", 4, 4, 0), ("grad", 3, 7, 1), ("curl", 3, 3, 0), ("div", 3, 3, 0), ("curl", 2, 4, 1)]


@pytest.mark.parametrize("space,n,p,prec", CASES)
def test_graph_solve_matches_eager(rz, ctx, space, n, p, prec):
    print(f"graph solve {space} n={n} p={p} prec={prec}", flush=True)
    a = synth.cell_coefficients(n ** 3, 1) if space == "grad" else 1.0
    pe = rz.Problem(ctx, n, p, a, 1.0, space=space, precision=prec)
    pg = rz.Problem(ctx, n, p, a, 1.0, space=space, precision=prec, graph=1)
    try:
        b = rhs(pe, [3])
        xe = torch.zeros_like(b)
        ie = pe.solve(b, xe)
        xg = torch.full_like(b, 7.0)
        for rep in range(3):   # capture, replay, and a new x vector (captured again)
            if rep == 2:
                xg = torch.zeros_like(b)
            ig = pg.solve(b, xg)
            torch.cuda.synchronize()
            assert ig.iters == ie.iters
            assert torch.equal(xg, xe), f"solve {rep} differs"
        assert ie.iters >= 2
        assert ie.rel_res <= 1e-8 and ig.rel_res == ie.rel_res
        cap, rep, seg = pg.graph_stats()
        # iterations 1.. of each solve ran from graphs, captured once per parity and x
        assert rep == 3 * (ie.iters - 1), (cap, rep, seg)
        assert cap == min(2, ie.iters - 1) * 2, (cap, rep, seg)
        assert seg == (2 if space == "grad" else 1)
        assert pe.graph_stats() == (0, 0, 0)
    finally:
        pe.close()
        pg.close()


@pytest.mark.parametrize("space", ["grad", "curl"])
def test_graph_multi_rhs_and_regrow(rz, ctx, space):
    print(f"graph multi-rhs {space}", flush=True)
    n, p = (3, 5) if space == "grad" else (2, 4)
    pe = rz.Problem(ctx, n, p, 1.0, 1.0, space=space)
    pg = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, graph=1)
    try:
        for nrhs in (2, 4, 2):   # 4 after 2 replaces the multi-vector buffers
            b = rhs(pe, list(range(10, 10 + nrhs)))
            xe = torch.zeros_like(b)
            xg = torch.zeros_like(b)
            ie = pe.solve(b, xe)
            ig = pg.solve(b, xg)
            torch.cuda.synchronize()
            assert [i.iters for i in ig] == [i.iters for i in ie]
            assert torch.equal(xg, xe)
            assert max(i.rel_res for i in ig) <= 1e-8
        assert pg.graph_stats()[1] > 0
    finally:
        pe.close()
        pg.close()


def test_graph_batched_matches_eager(rz):
    print("graph batched", flush=True)
    streams = [torch.cuda.Stream() for _ in range(2)]
    ctxs = [rz.Context(0, s) for s in streams]
    specs = [("grad", 3, 4), ("curl", 2, 3), ("div", 2, 4), ("grad", 2, 6), ("curl", 3, 2)]
    pe, pg, bs = [], [], []
    try:
        for i, (space, n, p) in enumerate(specs):
            pe.append(rz.Problem(ctxs[i % 2], n, p, 1.0, 1.0, space=space))
            pg.append(rz.Problem(ctxs[i % 2], n, p, 1.0, 1.0, space=space, graph=1))
            bs.append(rhs(pe[-1], [4 * i, 4 * i + 1]))
        torch.cuda.synchronize()
        xe = [torch.zeros_like(b) for b in bs]
        ie = rz.solve_batched(pe, bs, xe)
        for rep in range(2):
            xg = [torch.zeros_like(b) for b in bs]
            ig = rz.solve_batched(pg, bs, xg)
            torch.cuda.synchronize()
            for k in range(len(specs)):
                assert [i.iters for i in ig[k]] == [i.iters for i in ie[k]]
                assert torch.equal(xg[k], xe[k]), f"problem {k} replay {rep}"
        assert all(q.graph_stats()[1] > 0 for q in pg)
    finally:
        for q in pe + pg:
            q.close()
        for c in ctxs:
            c.close()
