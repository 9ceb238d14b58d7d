"""CPU oracle for the p-multigrid Riesz-map solver (Brubeck & Farrell,
"Multigrid solvers for the de Rham complex with optimal complexity in polynomial
degree").

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 NumPy/SciPy code written from the
paper's definitions; it shares no code, tables or constants with the HIP library
under ``paper_2211_14284_amd`` and neither imports the other.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.

Modules
  tables1d  -- 1-D FDM element: GLL nodes, eigenbasis, mass/stiffness, DP basis,
               differentiation matrix, broken basis (Sec. 2.2, 2.3, 3.2)
  lattice   -- degree-of-freedom numbering of Q_p / NCE_p / NCF_p on structured
               hexahedral meshes, Dirichlet masks (Sec. 2.4, 3.1)
  assemble  -- assembled global operators (Sec. 3.1-3.2, eq. sum-factorization)
  matfree   -- matrix-free sum-factorised apply (Sec. 3.2, Sec. 5)
  auxop     -- auxiliary sparse operator (eq. sum-factorization_approx)
  schwarz   -- static condensation, vertex-star patches, incomplete Cholesky on
               the static-condensation pattern, patch relaxation (Sec. 4.3-4.5)
  pmg       -- p-transfer, coarse problem, V(1,1) cycle and PCG (Sec. 4.3, 5)
  learned   -- least-squares separable fit to the broken diagonals, per-cell
               features, a hand-written NumPy MLP (forward, backward, Adam)
  hodge     -- mixed Hodge Laplacians k = 1, 2, 3: block system, Chebyshev-accelerated
               Riesz-map block preconditioner, preconditioned MINRES (Sec. 5.3)
  quadrature-- Gauss-Lobatto rules, sampled (triquadratic) coefficients and the
               cell-averaged separable auxiliary weights for trilinear cells

Readings of the paper where it is silent are listed in each function's docstring.
"""
