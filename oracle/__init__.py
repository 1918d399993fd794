"""Oracle: a plain, slow, CPU float64 implementation of the preconditioned
solve, written from the paper (Bonev & Hesthaven, "A hierarchical
preconditioner for wave problems in quasilinear complexity").

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  It shares no code with the
HIP library under ``paper_2105_07791_amd``; the only common inputs are the
seeded arrays produced by ``synth``.

Modules
  fem        P1 Galerkin assembly of the Helmholtz operator (Sec. 4.2, eq. 4.2)
  nd         box nested dissection, elimination tree, cluster trees (Sec. 3.1-3.3)
  exact      exact multifrontal LDR elimination and its inverse (eqs. 3.2-3.5,
             Algorithm 3.1)
  krylov     restarted GMRES / flexible GMRES (eq. 1.2, Sec. 4)
  rng        counter-based Gaussian generator for the random sketches
  hss        HSS matrices, interpolative decomposition, adaptive randomized
             compression (Sec. 2.2-2.3, Algorithm A.1)
  approx     the approximate factorization P = LDR (Algorithm 3.4)
  adjoint    adjoint gradient of a misfit through x = A(s)^-1 b
"""
