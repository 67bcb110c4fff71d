"""FP64 CPU oracle for the per-macro-element local work of one Newton step
of the entropy-variable macro-element HDG method.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check of
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
or call it.  The HIP library never does, and shares no code with it: the
two see the same seeded inputs (``paper_2507_22195_amd.workloads``) and
nothing else.

Plain, slow, obviously correct: dense numpy tables, quadrature written as
weighted sums, exact pointwise Jacobians from forward-mode dual numbers,
static condensation with explicit dense solves (LAPACK through numpy).

Modules
  ad        forward-mode dual numbers
  basis     2x2x2 Q_p macro space, Gauss quadrature, trace space
  physics   u(v), fluxes F, G, the EC / ES / KEPES trace fluxes, entropy
  local     residual, Jacobian blocks, condensation (R1-R6), recovery
  linearized  Jacobian-vector and vector-Jacobian products of the residual
  global_solve  the global trace system
  tet       tetrahedral macro-elements: 8 P_p sub-tetrahedra, simplex
            quadrature, affine geometry
  forms     residual, Jacobian and condensation on any macro shape given as
            quadrature tables (tetrahedral and hexahedral)

Every function is pinned by a CPU test (``tests/test_oracle_*.py``)
against identities the paper proves, closed forms, finite differences or
brute force; none is marked parity-unpinned.
"""
from . import ad, basis, physics, local  # noqa: F401
