"""CPU FP64 oracle for subdomain-deflated, block-local AMG Krylov solves.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method of Demidov & Rossi, "Subdomain
deflation combined with local AMG" (arXiv:1710.03940).  It exists to check
the GPU library; only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it.  It shares no code with the GPU library: neither
imports the other, and they meet only through the seeded inputs of the
`workloads` package.

Contents (each module cites the passages it follows):

* `deflation` - deflation basis Z, AZ, E = Z^T A Z and its exact FP64
  factorisation, the projector P = I - A Z E^{-1} Z^T and the solution
  recovery x = y + Z lambda (section "Subdomain deflation", eqs. (2)-(8),
  section "Implementation", projector equation), the inexact coarse solve
  and the deflation combined multiplicatively with a preconditioner of the
  original system (section "On precision of the coarse system solution");
* `sa` - per-subdomain smoothed-aggregation hierarchy with SPAI-0 or damped
  Jacobi smoothing (sections "Implementation" and "Benchmarks");
* `vcycle` - one V(1,1) cycle and the block-diagonal (non-overlapping local)
  preconditioner;
* `krylov` - deflated preconditioned CG, BiCGStab and BiCGStab(ell), and
  restarted flexible GMRES on the original system;
* `solver` - setup + solve with the library's calling conventions.

Readings of points the paper leaves open are listed in each module and in the
design notes of the repository.  Every function here is pinned by the CPU
tests (tests/test_oracle_pins.py, tests/test_oracle_fgmres.py) against facts that do not come from the
oracle itself; none is marked "parity unpinned".
"""
from .solver import OracleSolver, OracleParams, OracleError

__all__ = ["OracleSolver", "OracleParams", "OracleError"]
