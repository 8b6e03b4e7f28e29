"""Linear solves for the inner Newton step (Sec. III-A).

``dense_lu_solve`` is Gaussian elimination with partial pivoting written out
step by step, for brute-force checks on small systems.  ``sparse_solve`` calls
SciPy's SuperLU, the sparse direct solver family the paper uses; the Jacobian
pattern is structurally symmetric, so the minimum-degree ordering on A^T + A is
used for the fill-reducing column permutation.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class SingularError(ArithmeticError):
    pass


def dense_lu_solve(A, b):
    A = np.array(A, dtype=np.result_type(A, b, np.float64), copy=True)
    x = np.array(b, dtype=A.dtype, copy=True)
    n = A.shape[0]
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        if A[p, k] == 0:
            raise SingularError(f"zero pivot in column {k}")
        if p != k:
            A[[k, p]] = A[[p, k]]
            x[[k, p]] = x[[p, k]]
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    for i in range(n):  # L y = P b (unit lower)
        x[i] -= A[i, :i] @ x[:i]
    for i in range(n - 1, -1, -1):  # U x = y
        x[i] = (x[i] - A[i, i + 1:] @ x[i + 1:]) / A[i, i]
    return x


def sparse_solve(J, b):
    J = sp.csc_matrix(J)
    try:
        lu = spla.splu(J, permc_spec="MMD_AT_PLUS_A")
    except RuntimeError as exc:  # SuperLU reports exact singularity this way
        raise SingularError(str(exc)) from exc
    x = lu.solve(np.asarray(b))
    if not np.all(np.isfinite(x)):
        raise SingularError("non-finite solution")
    return x


def solve(J, b, method):
    if method == "dense":
        return dense_lu_solve(J.toarray() if sp.issparse(J) else J, b)
    return sparse_solve(J, b)
