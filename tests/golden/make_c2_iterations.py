"""Write c2_iterations.txt: the oracle's PCG iteration counts for the C2 recipe
(H(grad) Q_7 on n^3, cellwise alpha, beta log-uniform in [1e-2, 1e2) from seeds 1
and 2, U[-1,1) right-hand side from seed 0, Dirichlet boundary) at reduced sizes,
with the oracle alone (SC-PAFW relaxation with IC on the static-condensation
pattern, p-multigrid to Q_1, damping from 10 Lanczos steps, 2-norm criterion 1e-8).

  python tests/golden/make_c2_iterations.py [n ...]      (default: 8 16)

The library's iteration counts at the same sizes are compared with these within
one iteration (tests/test_gpu_c2_iterations.py).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth                                                    # noqa: E402
from oracle.lattice import Mesh, Lattice                        # noqa: E402
from oracle import assemble as asm, auxop, schwarz, pmg         # noqa: E402


def count(n, p=7):
    al, be = synth.cell_coefficients(n ** 3, 1), synth.cell_coefficients(n ** 3, 2)
    m = Mesh(n, n, n)
    lat, latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be))
    R = schwarz.SCRelaxGrad(lat, auxop.separable_operator(lat, auxop.cartesian_coefficient_array(lat, al, be)))
    Pr = pmg.prolongation(lat, latc)
    cs = pmg.CoarseSolver(latc, asm.with_dirichlet(latc, asm.cartesian_operator(latc, al, be)))
    mask = lat.dirichlet_mask()
    v0 = np.where(mask, 0.0, synth.uniform_pm1(99, lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    om = pmg.omega_from_lambda(lam)
    b = np.where(mask, 0.0, synth.rhs_values(lat.ndofs, 0))
    _, it, hist = pmg.pcg(A, b, pmg.VCycle(lat, A, R, Pr, cs, om))
    return it, om, hist[-1] / hist[0]


if __name__ == "__main__":
    sizes = [int(a) for a in sys.argv[1:]] or [8, 16]
    lines = ["# Oracle PCG iterations for the C2 recipe at reduced sizes (Q_7; cellwise alpha,",
             "# beta log-uniform in [1e-2, 1e2), seeds 1, 2; right-hand side seed 0; 2-norm",
             "# criterion 1e-8).  Written by make_c2_iterations.py (oracle only).",
             "# Columns: n, iterations, omega, final relative residual (recurrence)."]
    for n in sizes:
        t0 = time.time()
        it, om, rr = count(n)
        lines.append(f"{n} {it} {om:.12e} {rr:.3e}")
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "c2_iterations.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
