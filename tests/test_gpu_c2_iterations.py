"""PCG iteration counts of the H(grad) recipe against the oracle at reduced sizes.

Q_7 on n^3 cells (n = 8, 16), cellwise alpha and beta log-uniform in [1e-2, 1e2)
(seeds 1 and 2), U[-1,1) right-hand side (seed 0), Dirichlet boundary, FP64
protocol: the library and the oracle run the same method (SC-PAFW relaxation with IC
on the static-condensation pattern, hybrid V(1,1) to Q_1, damping from 10 Lanczos
steps seeded alike, PCG to the 2-norm criterion 1e-8; Sec. 5 and Table hgrad-iter).
Rounding differs between the two (summation order in the apply, the patch solves
and the dot products), so a count may move by one; it may not move by more.
The oracle's counts are in tests/golden/c2_iterations.txt (written by
tests/golden/make_c2_iterations.py from the oracle alone).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P = 7
HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    out = {}
    with open(os.path.join(HERE, "golden", "c2_iterations.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, it, om, _ = line.split()
            out[int(n)] = (int(it), float(om))
    return out


@pytest.fixture(scope="module")
def rz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14284_amd import rz as mod
    return mod


@pytest.fixture(scope="module")
def ctx(rz):
    return rz.Context(0, torch.cuda.current_stream())


@pytest.mark.parametrize("n", [8, 16])
def test_c2_iterations_match_oracle(rz, ctx, n):
    g = golden()
    if n not in g:
        pytest.skip(f"no oracle count for n = {n}")
    it_ref, om_ref = g[n]
    print(f"C2 iterations n={n}", flush=True)
    al = synth.cell_coefficients(n ** 3, 1)
    be = synth.cell_coefficients(n ** 3, 2)
    pb = rz.Problem(ctx, n, P, al, be)
    try:
        from oracle.lattice import Mesh, Lattice
        mask = Lattice(Mesh(n, n, n), "grad", P).dirichlet_mask()
        b = torch.as_tensor(np.where(mask, 0.0, synth.rhs_values(pb.ndofs, 0)), device="cuda:0")
        x = torch.empty_like(b)
        info = pb.solve(b, x)
        print(f"n={n}: library {info.iters} (omega {info.omega:.6e}), oracle {it_ref} (omega {om_ref:.6e})",
              flush=True)
        # the damping comes from the same 10 Lanczos steps on the same start vector
        assert abs(info.omega - om_ref) <= 1e-6 * om_ref
        assert abs(info.iters - it_ref) <= 1
        assert info.rel_res <= 1e-8
    finally:
        pb.close()
