"""Result record shared by the oracle's Newton loops."""

import dataclasses

import numpy as np

CONVERGED, MAXITER, DIVERGED, SINGULAR, LINEAR_FAIL = 0, 1, 2, 3, 4


@dataclasses.dataclass
class OracleResult:
    status: int
    iters: int                 # linear solves performed
    V: np.ndarray              # complex128 voltages of every bus / phase-node
    history: list              # max-norm of the mismatch before each step
    steps: list                # max |dx| of each Newton step (the paper's stop test)
    mismatch_inf: float        # max-norm of the final mismatch
    linear_iters: list = dataclasses.field(default_factory=list)  # Krylov steps per Newton step
    lu_fallback: bool = False  # a Krylov step failed and direct solves finished the iteration
    q_gen: np.ndarray = None   # three-phase: generator Q per phase-node (PV nodes solved for)

    @property
    def vm(self):
        return np.abs(self.V)

    @property
    def va(self):
        return np.angle(self.V)
