"""CPU FP64 oracle for DG acoustics on vertex-mapped pyramids.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP path; the only
common inputs are the seeded generators in ``synth``.

It is written to be plain, slow and checkable against the paper by eye:

* ``rules``    -- Gauss-Legendre / Gauss-Jacobi rules and the collapsed volume
                  and face cubatures (Section 4.1, minimal rule).
* ``basis``    -- the semi-nodal basis phi_ijk of Lemma 3 and its derivatives.
* ``geometry`` -- Bedrosian's vertex functions and the vertex map (Section 2).
* ``dg``       -- the semi-discrete acoustic DG right-hand side of Section 4.3,
                  with every element mass matrix assembled by quadrature and
                  inverted through an LU factorisation, plus projection, L2
                  error and energy.
* ``advection``-- the semi-discrete advection DG right-hand side of
                  Section 4.1 (upwind / central flux, periodic cubes).
* ``adjoint``  -- the discrete adjoint of the acoustic LSRK stepping.
* ``lsrk``     -- the low-storage RK(5,4) time stepper (Section 4.1,
                  Algorithm 3), coefficients of Carpenter and Kennedy.

Pins for every function live in ``tests/test_oracle_*.py``.  Functions without
an independent pin say "parity unpinned" in their docstring.
"""

from .dg import AcousticDG
from .lsrk import LSRK_A, LSRK_B, LSRK_C, lsrk_run

__all__ = ["AcousticDG", "LSRK_A", "LSRK_B", "LSRK_C", "lsrk_run"]
