"""Plain CPU FP64 oracle for the randomized DOT inversion hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
never does.  It shares no code with the HIP library: it is written from the
paper's definitions (Sections 2 and 3) with numpy/scipy, in FP64, slow and
direct on purpose.

Modules
  discretization  cell-centred finite-volume operator A(p) (Section 2, eq. PDE)
  pals            PaLS level set, smoothed Heaviside absorption, d mu / d p
  solvers         banded Cholesky, SuperLU, plain Jacobi-PCG
  estimators      simultaneous sources/detectors, sampled misfit, Jacobian,
                  gradient (Section 3.1, eqs. Rw, defW, defV, EsTResidual,
                  Jacobian kth column, UnbiasedGrad)
  design          Alg. 1 (optimized sources/detectors, HOOI/Tucker2) and the
                  complementary random sources/detectors (Section 3.2)

Pins: every function is checked in the ``-m "not gpu"`` tests against
closed forms, library special cases (DST-II), manufactured solutions,
finite differences, exact enumeration of expectations and the paper's
theorems.  Readings of silent or ambiguous passages are listed where they
are used.
"""

from . import design, discretization, estimators, pals, solvers  # noqa: F401
