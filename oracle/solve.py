"""GENP, triangular solves, the full RBT solve, backward error, iterative
refinement and the adjoint.  ORACLE: test infrastructure only.

The method (Eq. 1 and the three steps listed under it): transform A~ = U^T A V
and b~ = U^T b, solve A~ x~ = b~ by Gaussian elimination with no pivoting,
then x = V x~.

Readings:
  * a zero pivot is not perturbed: the elimination continues with IEEE
    Inf/NaN and `info` records the first exact zero pivot (1-based);
  * Eq. 7 is defined for one right-hand side; for several, it is taken per
    column and the maximum is reported;
  * refinement (Sec. 5) is the stationary one: x += V (LU)^-1 U^T (b - A x),
    stopping when the backward error reaches `tol` or after `max_iter` steps.

Parity: GENP is pinned by L U = A~ reconstruction, by exact rational
elimination at tiny n (Theorem 3) and by the growth bound Eq. 5; the solve by
exact rational solves at n <= 16 and the `orthog` closed-form inverse; the
backward error by the same closed form; the adjoint by a dense inverse and
central finite differences.  Refinement iteration counts: parity unpinned
(the paper prints none for these inputs).
"""
import numpy as np

from . import transform


def genp_unblocked(A):
    """Right-looking (kji) elimination without pivoting.

    Returns (LU, info): unit-lower L strictly below the diagonal, U on and
    above it, info = first k (1-based) with an exactly zero pivot, else 0.
    """
    LU = np.array(A, dtype=np.float64, copy=True)
    n = LU.shape[0]
    info = 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for k in range(n):
            p = LU[k, k]
            if p == 0.0 and info == 0:
                info = k + 1
            LU[k + 1:, k] /= p
            LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, info


def genp_blocked(A, nb=256, max_panels=None):
    """Same elimination as genp_unblocked, grouped in column panels of width
    nb so the trailing update is one matrix product per panel; it differs from
    the unblocked form only in the order of the roundings.
    max_panels: stop after that many panels (the factors are then those of
    the first max_panels * nb columns and the untouched Schur complement; used
    only to time a sample of the elimination).
    """
    LU = np.array(A, dtype=np.float64, copy=True)
    n = LU.shape[0]
    info = 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for k0 in range(0, n if max_panels is None else min(n, max_panels * nb), nb):
            k1 = min(k0 + nb, n)
            # eliminate inside the panel columns k0..k1-1 (all rows below)
            for k in range(k0, k1):
                p = LU[k, k]
                if p == 0.0 and info == 0:
                    info = k + 1
                LU[k + 1:, k] /= p
                LU[k + 1:, k + 1:k1] -= np.outer(LU[k + 1:, k], LU[k, k + 1:k1])
            if k1 < n:
                # U12 = L11^-1 A12 by forward substitution (unit L11)
                for k in range(k0, k1):
                    LU[k + 1:k1, k1:] -= np.outer(LU[k + 1:k1, k], LU[k, k1:])
                # Schur complement A22 -= L21 U12
                LU[k1:, k1:] -= LU[k1:, k0:k1] @ LU[k0:k1, k1:]
    return LU, info


def genp(A, nb=None):
    n = np.asarray(A).shape[0]
    if nb is None:
        nb = 0 if n < 2048 else 256
    return genp_blocked(A, nb) if nb else genp_unblocked(A)


def forward_unit_lower(LU, B):
    """Solve L Y = B with L the unit lower triangle of LU (column sweeps)."""
    Y = np.array(B, dtype=np.float64, copy=True)
    vec = Y.ndim == 1
    if vec:
        Y = Y[:, None]
    n = LU.shape[0]
    for j in range(n):
        Y[j + 1:] -= np.outer(LU[j + 1:, j], Y[j])
    return Y[:, 0] if vec else Y


def backward_upper(LU, Y):
    """Solve U X = Y with U the upper triangle of LU (column sweeps)."""
    X = np.array(Y, dtype=np.float64, copy=True)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    n = LU.shape[0]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for j in range(n - 1, -1, -1):
            X[j] /= LU[j, j]
            X[:j] -= np.outer(LU[:j, j], X[j])
    return X[:, 0] if vec else X


def forward_upper_transposed(LU, G):
    """Solve U^T Z = G (U^T is lower triangular, non-unit)."""
    Z = np.array(G, dtype=np.float64, copy=True)
    vec = Z.ndim == 1
    if vec:
        Z = Z[:, None]
    n = LU.shape[0]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for j in range(n):
            # row j of U^T is column j of U: sum_{i<j} U[i, j] Z[i] + U[j, j] Z[j]
            Z[j] = (Z[j] - LU[:j, j] @ Z[:j]) / LU[j, j]
    return Z[:, 0] if vec else Z


def backward_unit_lower_transposed(LU, Z):
    """Solve L^T W = Z (L^T is upper triangular with unit diagonal)."""
    W = np.array(Z, dtype=np.float64, copy=True)
    vec = W.ndim == 1
    if vec:
        W = W[:, None]
    n = LU.shape[0]
    for j in range(n - 1, -1, -1):
        # row j of L^T is column j of L below the diagonal
        W[j] = W[j] - LU[j + 1:, j] @ W[j + 1:]
    return W[:, 0] if vec else W


def lu_solve(LU, B):
    return backward_upper(LU, forward_unit_lower(LU, B))


def rbt_solve(A, B, U, V, d, nb=None, granule=1):
    """The method of Eq. 1: returns (X, LU of A~, info). granule: the
    reference size of the butterflies (structure.reference_size)."""
    At = transform.two_sided(A, U, V, d, granule)
    Bt = transform.apply_transpose_left(B, U, d, granule)
    LU, info = genp(At, nb)
    Xt = lu_solve(LU, Bt)
    X = transform.apply_left(Xt, V, d, granule)
    return X, LU, info


def rbt_solve_kind(A, B, U, V, d, kind="diag", granule=1, sides=2, nb=None):
    """The method of Eq. 1 with either butterfly kind (transform.transform_pair)
    and one or two sides (sides = 1: A~ = U^T A and x = x~, Sec. 7).
    Returns (X, LU of A~, info)."""
    fwd, undo = transform.transform_pair(kind)
    At = transform.two_sided_kind(A, U, V, d, kind, granule, sides)
    Bt = fwd(B, U, d, granule)
    LU, info = genp(At, nb)
    Xt = lu_solve(LU, Bt)
    X = Xt if sides == 1 else undo(Xt, V, d, granule)
    return X, LU, info


def backward_error(A, X, B):
    """Eq. 7, infinity norms, per column; returns the maximum over columns."""
    A = np.asarray(A, dtype=np.float64)
    X2 = np.asarray(X, dtype=np.float64).reshape(A.shape[0], -1)
    B2 = np.asarray(B, dtype=np.float64).reshape(A.shape[0], -1)
    R = B2 - A @ X2
    anorm = np.abs(A).sum(axis=1).max()
    num = np.abs(R).max(axis=0)
    den = anorm * np.abs(X2).max(axis=0) + np.abs(B2).max(axis=0)
    return float((num / den).max())


def refine(A, B, X, LU, U, V, d, tol, max_iter):
    """Stationary refinement (Sec. 5) with the RBT-transformed factors.

    Returns (X, iterations, backward error).  Each step: R = B - A X,
    D = V (LU)^-1 U^T R, X += D.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    it = 0
    be = backward_error(A, X, B)
    while be > tol and it < max_iter:
        R = np.asarray(B) - A @ X
        D = transform.apply_left(lu_solve(LU, transform.apply_transpose_left(R, U, d)), V, d)
        X += D
        it += 1
        be = backward_error(A, X, B)
    return X, it, be


def adjoint(LU, X, G, U, V, d):
    """Gradients of a loss L(X) with dL/dX = G for X = A^-1 B.

    lambda = A^-T G = U A~^-T V^T G  (A = U^-T A~ V^-1), with A~^T = U_f^T L^T:
    solve U_f^T Z = V^T G, then L^T W = Z, and lambda = U W.
    Returns (dA, dB) = (-lambda X^T, lambda).
    """
    Gh = transform.apply_transpose_left(G, V, d)
    Z = forward_upper_transposed(LU, Gh)
    W = backward_unit_lower_transposed(LU, Z)
    lam = transform.apply_left(W, U, d)
    lam2 = lam.reshape(LU.shape[0], -1)
    X2 = np.asarray(X).reshape(LU.shape[0], -1)
    return -lam2 @ X2.T, lam
