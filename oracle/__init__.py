"""FP64 CPU oracle of the P1-P1 IPCS (incremental pressure correction,
Adams-Bashforth/Crank-Nicolson convection) time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the HIP library is checked against.  Only the test
suite, the package smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never routes through it.  It shares no code with
the HIP library: the only common inputs come from the seeded generators in
``synth/``.

Modules
  p1          element geometry, closed-form P1 element matrices, assembly
  quadrature  Gauss-Legendre rules collapsed onto simplices (pins, norms)
  krylov      Jacobi-preconditioned CG and BiCGStab (textbook loops)
  ipcs        setup + one time step following the paper's Alg. 1/Alg. 2
  naive       per-cell quadrature reassembly of the tentative system
  graph       CSR pattern, Cuthill-McKee ordering, greedy cell colouring
  mixed       FP32-inner / FP64-outer iterative refinement
  mpnn        message-passing warm-start network, forward/backward/Adam
  amg         smoothed-aggregation multigrid hierarchy, V-cycle, AMG-PCG

Readings of the paper where it is silent or inconsistent are listed in the
docstrings of the functions that take them.
"""
