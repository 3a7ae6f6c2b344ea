"""Plain FP64 CPU oracle for the spin-charge Krylov kernel.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, calls or
links this code; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do. It shares no code with the HIP path: it is written in
numpy/scipy, un-fused and in the order of the paper's definitions, so that
it can be checked against the paper by eye.

Modules
  fermi      Fermi occupations, divided differences, chemical potential
  expansion  congruence factor Z, eigenbasis of H-perp, ground-state map q[n]
  response   directional derivative dq[n + lambda v]/dlambda (first order)
  krylov     preconditioned low-rank Krylov kernel (K0 J)^-1 K0 delta
  mulliken   Mulliken projection of a density-matrix change

Every function is pinned by tests in tests/test_oracle_pins.py against
something other than itself (finite differences of the full map, an
arbitrary-precision brute force, closed forms, invariants, GMRES and dense
linear algebra). Parity is unpinned only where the paper's own model data
are missing (its Fe parameterization and figures); see the module docs.
"""

from .fermi import divided_difference_matrix, solve_mu  # noqa: F401
from .expansion import (congruence_lowdin, congruence_cholesky, spin_hamiltonians,  # noqa: F401
                        expansion_point, q_of_n)
from .response import response, response_potentials  # noqa: F401
from .krylov import kernel_apply, jacobian_exact  # noqa: F401
from .mulliken import mulliken  # noqa: F401
