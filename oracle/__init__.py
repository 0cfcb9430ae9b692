"""FP64 CPU oracle for the spectral split-step Pade (SSSP) range march.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct reference
that the HIP library is checked against.  Only tests/, the smoke check in
__graft_entry__.py and the CPU-baseline leg of bench.py may import it.  It shares no code
with the library (no kernels, tables, helpers or headers); both receive their inputs from
the seeded generators in workloads/.

Modules:
  pade       Pade coefficients in 60-digit arithmetic (Sec. 2; Algorithm 1, first step)
  dst        orthonormal DST-I (Sec. 3.1) and its O(N^2) definition
  bases      grids, eigenvalues and transforms of the Dirichlet, Neumann and periodic
             boundary conditions (Sec. 3.1)
  modal      normal-mode starter and normal-mode field (Sec. 3.2)
  sssp       the range march in sum and product form (Sec. 3, eq. neumannseries, Alg. 1)
  reference  closed-form and brute-force references used to pin the oracle itself

Every function here is pinned by tests in tests/test_oracle_*.py to facts fixed by the
paper or by mathematics (Pade matching order, unitarity of the standard approximant,
the normal-mode sum of a homogeneous Dirichlet waveguide, dense eigendecomposition of X
on tiny grids, norm conservation, the M = 0 isovelocity special case).
"""
from .pade import pade, PadeCoeffs, taylor_coefficients
from .dst import dst, idst, dst_matrix, dst_direct
from .sssp import Plan, MarchResult, transmission_loss, OK, NOT_CONVERGED, DIVERGED

__all__ = ["pade", "PadeCoeffs", "taylor_coefficients", "dst", "idst", "dst_matrix",
           "dst_direct", "Plan", "MarchResult", "transmission_loss", "OK",
           "NOT_CONVERGED", "DIVERGED"]
