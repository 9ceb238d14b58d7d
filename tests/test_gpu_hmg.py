"""Geometric h-multigrid on the Q_1 space as the coarse solver of the p-multigrid
cycle (rz_opts.coarse = RZ_COARSE_HMG, the h-hierarchy below p = 1 of Sec. 5.1)
against the oracle's HMGCoarse, through the C ABI.

The hierarchy (free vertices per level) must equal the oracle's; one cycle on a
coarse right-hand side and the whole p-multigrid V-cycle around it agree to 1e-12
relative (FP64 throughout, the sums in another order); the PCG iteration count is
the oracle's within one and the solve reaches a true relative residual of 1e-8.
Graph capture of the CG iterations needs no cut around this coarse solver (one
segment per iteration, bits equal to the eager solve).  Meshes whose coarsest level
exceeds 4096 free vertices are rejected.

H(curl)/H(div) (NCE_1/NCF_1 hierarchy with Hiptmair relaxation, the oracle's
HiptmairHMG): the hierarchy equals the oracle's, the p-multigrid V-cycle around it
agrees with the oracle's within the tolerance that the statically condensed
relaxation's own conditioning allows (as for the direct coarse solve), and with
alpha = beta = 1 the solve's iteration count is the oracle's within one."""
import numpy as np
import pytest

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, auxop, schwarz, pmg, hiptmair as hp

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


def rel(a, b):
    nb = max(np.linalg.norm(b), 1e-300)
    mb = max(np.abs(b).max(initial=0.0), 1e-300)
    return max(np.linalg.norm(a - b) / nb, np.abs(a - b).max(initial=0.0) / mb)


def T(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def coefs(n, seed=1):
    nc = int(np.prod(n))
    return synth.cell_coefficients(nc, seed), synth.cell_coefficients(nc, seed + 1)


class Ref:
    def __init__(self, n, p, al, be, dirichlet=0x3F, relax=True):
        m = Mesh(*n, dirichlet=dirichlet)
        self.lat, self.latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
        self.A0 = asm.with_dirichlet(self.latc, asm.cartesian_operator(self.latc, al, be))
        self.hmg = pmg.HMGCoarse(self.latc, self.A0, min_free=512)
        if relax:
            self.A = asm.with_dirichlet(self.lat, asm.cartesian_operator(self.lat, al, be))
            co = auxop.cartesian_coefficient_array(self.lat, al, be)
            self.R = schwarz.SCRelaxGrad(self.lat, auxop.separable_operator(self.lat, co))
            self.Pr = pmg.prolongation(self.lat, self.latc)


# one, two and three coarsenings; all-Dirichlet and mixed boundaries (the free box
# then holds a boundary plane on some sides); a mesh that is not coarsened at all
@pytest.mark.parametrize("n,dirichlet", [((16, 8, 8), 0x3F), ((32, 16, 16), 0x3F), ((16, 16, 8), 0x15),
                                         ((12, 12, 12), 0x2A), ((20, 12, 8), 0x3F), ((7, 9, 8), 0x3F)])
def test_hmg_coarse_solve_parity(rz, ctx, n, dirichlet):
    print(f"hmg coarse solve n={n} dir={dirichlet:#x}", flush=True)
    al, be = coefs(n)
    ref = Ref(n, 2, al, be, dirichlet, relax=False)
    pb = rz.Problem(ctx, n, 2, al, be, omega=0.3, dirichlet=dirichlet, coarse=rz.COARSE_HMG)
    try:
        assert pb.hmg_levels() == [a.shape[0] for a in ref.hmg.A]
        rc = np.where(ref.latc.dirichlet_mask(), 0.0, synth.uniform_pm1(31, ref.latc.ndofs))
        xc = torch.empty(pb.ncoarse, dtype=torch.float64, device="cuda:0")
        for _ in range(2):    # the level vectors hold the last call's values: no state carried over
            pb.coarse_solve(T(rc), xc)
            assert rel(H(xc), ref.hmg.solve(rc)) < 1e-12
    finally:
        pb.close()


@pytest.mark.parametrize("n,p,prec", [((16, 8, 8), 2, 0), ((12, 12, 12), 3, 0), ((16, 8, 8), 2, 1)])
def test_hmg_vcycle_and_solve(rz, ctx, n, p, prec):
    print(f"hmg vcycle/solve n={n} p={p} prec={prec}", flush=True)
    al, be = coefs(n, 3)
    ref = Ref(n, p, al, be)
    mask = ref.lat.dirichlet_mask()
    om = 0.37
    pb = rz.Problem(ctx, n, p, al, be, omega=om, precision=prec, coarse=rz.COARSE_HMG)
    try:
        V = pmg.VCycle(ref.lat, ref.A, ref.R, ref.Pr, ref.hmg, om)
        if prec == 0:
            r = np.where(mask, 0.0, synth.uniform_pm1(41, ref.lat.ndofs))
            z = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
            pb.vcycle(T(r), z)
            assert rel(H(z), V(r)) < 1e-12
        b = np.where(mask, 0.0, synth.rhs_values(ref.lat.ndofs, 0))
        _, it_ref, _ = pmg.pcg(ref.A, b, V)
        x = torch.zeros(pb.ndofs, dtype=torch.float64, device="cuda:0")
        info = pb.solve(T(b), x)
        xg = H(x)
        assert info.rel_res <= 1e-8
        assert np.linalg.norm(b - ref.A @ xg) <= 1e-8 * np.linalg.norm(b)
        assert abs(info.iters - it_ref) <= (1 if prec == 0 else 2), (info.iters, it_ref)
    finally:
        pb.close()


def test_hmg_graph_single_segment(rz, ctx):
    print("hmg graph", flush=True)
    n, p = (16, 8, 8), 3
    al, be = coefs(n, 5)
    pe = rz.Problem(ctx, n, p, al, be, coarse=rz.COARSE_HMG)
    pg = rz.Problem(ctx, n, p, al, be, coarse=rz.COARSE_HMG, graph=1)
    try:
        b = T(synth.rhs_values(pe.ndofs, 7))
        xe = torch.zeros_like(b)
        ie = pe.solve(b, xe)
        for _ in range(2):
            xg = torch.zeros_like(b)
            ig = pg.solve(b, xg)
            torch.cuda.synchronize()
            assert ig.iters == ie.iters and torch.equal(xg, xe)
        cap, rep, seg = pg.graph_stats()
        assert seg == 1 and rep == 2 * (ie.iters - 1)
    finally:
        pe.close()
        pg.close()


def test_hmg_large_solve_protocols(rz, ctx):
    """The C2 layout at Q_4 (32^3 cells, log-uniform cell coefficients): three
    coarsenings (29791, 3375, 343 free vertices); FP64, mixed and defect-correction
    protocols reach 1e-8."""
    print("hmg 32^3 Q_4", flush=True)
    n, p = 32, 4
    al, be = coefs((n, n, n), 1)
    its = {}
    for prec in (0, 1, 2):
        pb = rz.Problem(ctx, n, p, al, be, precision=prec, coarse=rz.COARSE_HMG)
        try:
            assert pb.hmg_levels() == [29791, 3375, 343]
            b = T(synth.rhs_values(pb.ndofs, 11))
            x = torch.zeros_like(b)
            info = pb.solve(b, x)
            assert info.rel_res <= 1e-8, (prec, info.rel_res)
            its[prec] = info.iters
        finally:
            pb.close()
    pd = rz.Problem(ctx, n, p, al, be)
    try:
        b = T(synth.rhs_values(pd.ndofs, 11))
        x = torch.zeros_like(b)
        idir = pd.solve(b, x).iters
    finally:
        pd.close()
    print("iterations hmg", its, "direct", idir, flush=True)
    assert its[0] <= 2 * idir


def test_hmg_rejections(rz, ctx):
    with pytest.raises(rz.RzError):   # 19 cells per axis: no coarsening, 18^3 > 4096 free vertices
        rz.Problem(ctx, 19, 1, 1.0, 1.0, coarse=rz.COARSE_HMG)
    with pytest.raises(rz.RzError):   # only with the statically condensed vector relaxation
        rz.Problem(ctx, 4, 2, 1.0, 1.0, space="curl", coarse=rz.COARSE_HMG, decomposition=rz.DECOMP_FULL,
                   patch_solver=rz.PATCH_CHOLESKY)
    with pytest.raises(rz.RzError):
        rz.Problem(ctx, 4, 2, 1.0, 1.0, coarse=7)


class RefVec:
    def __init__(self, space, n, p, al, be):
        m = Mesh(*n)
        self.lat, self.latc = Lattice(m, space, p), Lattice(m, space, 1)
        Araw = asm.cartesian_operator(self.lat, al, be)
        self.A = asm.with_dirichlet(self.lat, Araw)
        self.mask = self.lat.dirichlet_mask()
        self.R = hp.SCRelaxPH(self.lat, Araw, be)
        self.Pr = pmg.prolongation(self.lat, self.latc)
        A0 = asm.with_dirichlet(self.latc, asm.cartesian_operator(self.latc, al, be))
        self.hmg = pmg.HiptmairHMG(self.latc, A0, min_free=512)


# (8, 8, 4) cells: 532 free NCE_1 and 640 free NCF_1 DoFs, one coarsening
@pytest.mark.parametrize("space", ["curl", "div"])
@pytest.mark.parametrize("coef", ["unit", "cell"])
def test_hmg_vec_vcycle_parity(rz, ctx, space, coef):
    print(f"hmg vec vcycle {space} {coef}", flush=True)
    n, p = (8, 8, 4), 2
    al, be = coefs(n, 3) if coef == "cell" else (1.0, 1.0)
    ref = RefVec(space, n, p, al, be)
    om = 0.2
    pb = rz.Problem(ctx, n, p, al, be, space=space, omega=om, coarse=rz.COARSE_HMG)
    try:
        assert pb.hmg_levels() == [a.shape[0] for a in ref.hmg.A]
        V = pmg.VCycle(ref.lat, ref.A, ref.R, ref.Pr, ref.hmg, om)
        r = np.where(ref.mask, 0.0, synth.uniform_pm1(41, ref.lat.ndofs))

        class Noisy:        # the oracle relaxation with 1e-12 relative output noise
            k = 0

            def apply(self, x):
                Noisy.k += 1
                y = ref.R.apply(x)
                return y * (1 + 1e-12 * synth.uniform_pm1(100 + Noisy.k, y.size))
        z0 = V(r)
        amp = np.linalg.norm(pmg.VCycle(ref.lat, ref.A, Noisy(), ref.Pr, ref.hmg, om)(r) - z0) / np.linalg.norm(z0)
        tol = max(1e-11, 50 * amp)
        z = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
        pb.vcycle(T(r), z)
        zg = H(z)
        zg[ref.mask] = 0.0
        assert rel(zg, z0) < tol, (rel(zg, z0), tol)
    finally:
        pb.close()


@pytest.mark.parametrize("space", ["curl", "div"])
def test_hmg_vec_solve(rz, ctx, space):
    print(f"hmg vec solve {space}", flush=True)
    n, p = (8, 8, 4), 2
    ref = RefVec(space, n, p, 1.0, 1.0)
    mask = ref.mask
    v0 = np.where(mask, 0.0, synth.uniform_pm1(99, ref.lat.ndofs))
    om = pmg.omega_from_lambda(pmg.lanczos_lambda_max(ref.A, lambda r: np.where(mask, 0.0, ref.R.apply(r)), v0))
    pb = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, coarse=rz.COARSE_HMG)
    pg = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, coarse=rz.COARSE_HMG, graph=1)
    try:
        assert abs(pb.omega() - om) < 1e-6 * om
        b = np.where(mask, 0.0, synth.rhs_values(ref.lat.ndofs, 0))
        _, it_ref, _ = pmg.pcg(ref.A, b, pmg.VCycle(ref.lat, ref.A, ref.R, ref.Pr, ref.hmg, om))
        x = torch.zeros(pb.ndofs, dtype=torch.float64, device="cuda:0")
        info = pb.solve(T(b), x)
        xg = H(x)
        assert info.rel_res <= 1e-8
        assert np.linalg.norm(b - ref.A @ xg) <= 1e-8 * np.linalg.norm(b)
        assert abs(info.iters - it_ref) <= 1, (info.iters, it_ref)
        xr = torch.zeros_like(x)
        ig = pg.solve(T(b), xr)
        assert ig.iters == info.iters and torch.equal(xr, x)
    finally:
        pb.close()
        pg.close()


def test_hmg_vec_c3_layout(rz, ctx):
    """NCE_6 and NCF_6 on 16^3 (alpha = beta = 1): three levels (10,800 / 1,176 / 108
    free NCE_1 DoFs), FP64 and mixed protocols reach 1e-8; iterations against the
    dense coarse inverse printed."""
    print("hmg vec 16^3 p=6", flush=True)
    for space in ("curl", "div"):
        its = {}
        for co in (rz.COARSE_DIRECT, rz.COARSE_HMG):
            for prec in (0, 1):
                pb = rz.Problem(ctx, 16, 6, 1.0, 1.0, space=space, precision=prec, coarse=co)
                try:
                    if co == rz.COARSE_HMG and space == "curl":
                        assert pb.hmg_levels() == [10800, 1176, 108]
                    b = T(synth.rhs_values(pb.ndofs, 11))
                    x = torch.zeros_like(b)
                    info = pb.solve(b, x)
                    assert info.rel_res <= 1e-8, (space, co, prec, info.rel_res)
                    its[(co, prec)] = info.iters
                finally:
                    pb.close()
        print(space, "iterations (coarse, precision)", its, flush=True)
        assert its[(rz.COARSE_HMG, 0)] <= its[(rz.COARSE_DIRECT, 0)] + 4
