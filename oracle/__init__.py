"""Plain FP64 CPU oracle for the closest point method (CPM) hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package. The library's product
path never calls it, and it shares no code with the library: every function
here is written from the paper (May, Haynes & Ruuth, "A closest point method
library for PDEs on surfaces with parallel domain decomposition solvers and
preconditioners", arXiv 2110.06322) and from the textbook definitions it
cites, in slow and obviously-checkable NumPy/SciPy.

Modules
  surfaces  closest point functions cp_S (Sec. 2.1, eq. cpFunc)
  band      active / ghost node sets Sigma_A, Sigma_G (Sec. 2.1)
  operator  extension E, neighbour sum, stabilized operator A (Sec. 2.1, eq. lapBel)
  krylov    restarted right-preconditioned (F)GMRES (Sec. 4.1.1: GMRES default)
  schwarz   partition, overlap, local problems, ILU(0), RAS / ORAS (Sec. 2.2)
  adjoint   A^T and gradients of a quadratic loss through the solve
  reaction  IMEX-Euler Gray-Scott step (Sec. 1, eq. rdsys; Sec. 4.1.5)

Pins (what fixes each part independently of itself) live in tests/test_oracle_*.py.
Parity unpinned: none of the paper's printed numbers (Tables 1-3) can be
reproduced here (torus radii, input files, ParMETIS partitions, hardware are
unavailable). The ORAS Robin lumping is a stated reading (no passage gives
its discrete form); the pins check that reading on a hand-worked case, by
the Robin substitution row by row, by its alpha -> infinity limit (RAS) and
by leaving the solution unchanged.
"""
