"""Sparse linear solve used by the oracle (test infrastructure).

At small eps the prediction system of (4.5) is ill-conditioned: in an
optically thick cell the isotropic mode sees only the small effective
absorption left over after the material coupling (4.5c) is substituted, so
rounding each matrix entry to binary64 already moves the solution in the
11th digit.  The oracle therefore assembles its systems in 80-bit extended
precision (numpy.longdouble) and solves them by classical iterative
refinement: an FP64 sparse LU supplies corrections, the residual is formed
in extended precision.  The result is the solution of the stated system to
well below 1e-14 relative, i.e. a reference that does not depend on how a
particular FP64 solver rounds.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

XP = np.longdouble  # extended precision used by the oracle's arithmetic


def coo(rows, cols, vals, n):
    """Assemble an n x n CSR matrix in extended precision from COO pieces."""
    r = np.concatenate([np.ravel(x) for x in rows]).astype(np.int64)
    c = np.concatenate([np.ravel(x) for x in cols]).astype(np.int64)
    v = np.concatenate([np.ravel(np.asarray(x, dtype=XP)) for x in vals])
    return sp.csr_matrix((v, (r, c)), shape=(n, n), dtype=XP)


def solve_refined(A, b, residual=None, max_refine=40):
    """Solve A x = b (A in extended precision) by LU + iterative refinement.

    `residual(x)`, when given, replaces b - A x (an algebraically identical
    evaluation); the FP64 LU of A only supplies corrections.  Refinement stops
    when the correction falls below 1e-19 relative or stops shrinking.

    Accuracy: the answer is exact for the extended-precision system up to its
    own sensitivity.  Far from equilibrium in very thick cells (ac*beta of
    (4.5c) above ~1e7) that sensitivity exceeds 1e8 and no 64- or 80-bit
    evaluation resolves the solution below ~1e-11; near-equilibrium states
    (the workloads) are resolved to ~1e-15.

    Returns (x in extended precision, number of refinement sweeps,
    final relative correction)."""
    A64 = sp.csc_matrix(A.astype(np.float64))
    lu = spla.splu(A64)
    b = np.asarray(b, dtype=XP)
    if residual is None:
        residual = lambda x: b - A @ x
    x = lu.solve(b.astype(np.float64)).astype(XP)
    rel = np.inf
    k = 0
    for k in range(1, max_refine + 1):
        r = residual(x)
        dx = lu.solve(r.astype(np.float64)).astype(XP)
        x = x + dx
        scale = np.max(np.abs(x)) if x.size else XP(1)
        prev, rel = rel, (float(np.max(np.abs(dx)) / scale) if scale > 0 else 0.0)
        if rel < 1e-19 or (k >= 4 and rel > 0.5 * prev):
            break
    return x, k, rel
