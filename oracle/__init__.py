"""CPU FP64 oracle for block PLHR (Vecharynski & Knyazev, arXiv:1408.0042).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this package; only the test-suite, the smoke check and the CPU baseline
leg of the benchmark do.  It shares no code with the HIP implementation: it
assembles operators as scipy.sparse matrices and solves the small projected
problems with LAPACK through scipy, in the order and notation of the paper.

Modules
  operators  sparse assembly of the model operators (FD Dirichlet, Bloch
             periodic, bilinear/trilinear finite elements) and a potential
  mg         geometric multigrid V-cycle used as the HPD preconditioner T,
             and the AV-MG / INV-MG preconditioners of Appendix A
             (Algorithms 4 and 5)
  plhr       Algorithms 1, 2 and 3 of the paper (single-vector PLHR, block
             PLHR in complex arithmetic, block PLHR in real arithmetic), the
             final Rayleigh-Ritz step and the convergence test
  hf         Hellmann-Feynman eigenvalue gradient with respect to a potential
  dense      brute-force dense reference: the k eigenpairs nearest sigma
"""
