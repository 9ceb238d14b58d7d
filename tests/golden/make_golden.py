"""Rewrite the two regression fixtures of this folder from the oracle alone.

  python tests/golden/make_golden.py

fdm_tables_appendix.txt: per p = 1..9, the 1-D FDM mass entries B_00, B_0p and the
generalised eigenvalues lambda_1..lambda_{p-1} (Sec. 2.2, eqs. fdmbasis-eigs).
vertex_patch_pattern_counts.txt: per p = 2..9, rows, lower non-zeros and the
largest row count of the static-condensation pattern of an interior vertex patch
(Sec. 4.4-4.5).  The numbers were first obtained by a scratch computation from
the paper's definitions made outside this repository; this script reproduces
them from ``oracle/`` (it calls nothing else), so the stored values come from a
committed script.  Closed forms pin part of them independently (tests).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.tables1d import Element1D          # noqa: E402
from oracle.lattice import Mesh, Lattice       # noqa: E402
from oracle import schwarz                     # noqa: E402


def tables():
    lines = ["# 1-D FDM tables (Sec. 2.2, eqs. fdmbasis, fdmdualbasis, unisolvence, eigs):",
             "# GLL nodes, exact GLL mass/stiffness, generalised eigenproblem.",
             "# Columns: p, B_00, B_0p, lambda_1 .. lambda_{p-1}.  Written by make_golden.py",
             "# (oracle only); first obtained by a scratch computation from the definitions",
             "# outside this repository.  Regression fixture: the closed forms for p <= 4",
             "# are asserted separately in test_oracle_tables.py."]
    for p in range(1, 10):
        el = Element1D(p)
        vals = [f"{el.B[0, 0]:.15f}", f"{el.B[0, p]:.15f}"] + [f"{v:.10f}".rstrip("0").rstrip(".")
                                                                for v in el.lam]
        lines.append(" ".join([str(p)] + vals))
    return lines


def pattern_counts():
    lines = ["# Interior H(grad) vertex-star interface patch on a Cartesian mesh (Sec. 4.4-4.5):",
             "# static-condensation sparsity pattern of S_v, derived symbolically from the",
             "# Kronecker structure of the auxiliary operator (1-D mass: diagonal + (0,p);",
             "# 1-D stiffness: diagonal + rows/columns 0 and p).  Columns: p, interface rows,",
             "# nnz(lower triangle incl. diagonal), max nnz per row.  Rows = 1 + 6(p-1) + 12(p-1)^2",
             "# and max = 6p - 5 by closed forms (asserted in the test); nnz is a regression value.",
             "# Written by make_golden.py (oracle only); first obtained by a scratch computation",
             "# from the definitions outside this repository."]
    for p in range(2, 10):
        lat = Lattice(Mesh(2, 2, 2), "grad", p)
        pat = schwarz.symbolic_schur_pattern_grad(lat)
        vid, dofs = [x for x in schwarz.vertex_patches_grad(lat) if x[0] == 13][0]
        pv = pat[dofs][:, dofs].toarray().astype(bool)
        lines.append(f"{p} {len(dofs)} {int(np.tril(pv).sum())} {int(pv.sum(1).max())}")
    return lines


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else HERE
    with open(os.path.join(out, "fdm_tables_appendix.txt"), "w") as f:
        f.write("\n".join(tables()) + "\n")
    with open(os.path.join(out, "vertex_patch_pattern_counts.txt"), "w") as f:
        f.write("\n".join(pattern_counts()) + "\n")
