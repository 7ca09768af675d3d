"""Plain FP64 CPU oracle for the matrix-free hyperelastic operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package: only the tests,
the smoke check and the CPU-baseline leg of the benchmark do. It shares no code with the HIP
library (no kernels, no headers, no tables); the only thing both sides see is the seeded input
generator in ``workloads``, which holds none of the method's arithmetic.

What it computes is the plain Galerkin definition that the matrix-free method reproduces up to
rounding order (Sections 2 and 6 of the paper: the same integrals, evaluated by quadrature):

* the residual r(v, u) = (Grad v, P)  with  P = F S,  S = 2 dPsi/dC          (Section 2, Eq. of the
  material residual; Section 3 for S);
* the linearised operator D_u r(v, du) = (Grad v, A : Grad du)  with A = dP/dF, built from the
  fourth-order tensor 4 d^2Psi/dCdC of the appendix (a *different* formulation than the
  directional-derivative action forms of Section 5 that the GPU kernels evaluate);
* explicit element matrices from dense basis tables (no sum factorisation), Gauss quadrature
  with p+1 points per direction, Lagrange elements on Gauss-Lobatto nodes.

Modules: ``basis`` (1D rules), ``mesh`` (structured hex lattices), ``material`` (energies,
stresses, tangent moduli), ``fem`` (geometry, residual, tangent, energy, transfers), ``fiber``
(fibre structure tensors), ``stability`` (80-digit stress and directional derivative for the
forward-stability study).

Parity status per function is listed in each module header. Every function here is pinned by a
``-m "not gpu"`` test in ``tests/test_oracle_*.py`` against something other than itself
(closed forms, finite/complex-step derivatives of the strain energy, patch and rigid-body
tests, the worked example of the fibre-parameter table).
"""

from . import basis, fiber, material, mesh, fem, stability  # noqa: F401
