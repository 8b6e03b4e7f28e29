"""Plain FP64 CPU oracle for the Newton power-flow iteration.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
GPU library never calls it and shares no code with it.

It follows the paper's equations step by step, in the paper's order:

* ``ybus``   - nodal admittance assembly (Sec. II, eq. 1-3; eq. 11 blocks),
  written independently of the input generator's stamping;
* ``polar``  - single-phase polar power flow (Sec. II-A, eq. 4-10 and the
  single-phase Newton-Raphson iteration table);
* ``cim``    - three-phase current-injection method (Sec. II-B, eq. 12-23 and
  the three-phase Newton-Raphson (CIM) iteration table);
* ``linalg`` - the linear solves of the inner step (Sec. III-A): a written-out
  dense LU with partial pivoting for small systems and SciPy's SuperLU (the
  library the paper uses) for large ones.

Every function is pinned by the CPU test suite against closed forms, finite
differences, power balance, an independent ladder (backward/forward sweep)
solution of radial feeders and brute force on tiny inputs.
"""

from .result import OracleResult, CONVERGED, MAXITER, DIVERGED, SINGULAR  # noqa: F401
from . import ybus, polar, cim, linalg  # noqa: F401
