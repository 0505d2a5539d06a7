"""Gaussian elimination with partial pivoting (GEPP), the robust solver of
the fallback in Sec. 5.  ORACLE: test infrastructure only (see
oracle/__init__.py).

Definition followed: at step k pick the row p >= k with the largest |a_pk|
(the first such row on ties), interchange rows k and p over the whole row,
record ipiv[k] = p + 1 (1-based, LAPACK's convention), then the multipliers
l_ik = a_ik / a_kk and the update a_ij -= l_ik a_kj for i, j > k.  The
result is P A = L U with the interchanges applied in order.  A zero pivot
column records info = k + 1 (first) and is not interchanged.

Parity: pinned against LAPACK's getrf/getrs (scipy.linalg.lu_factor /
lu_solve) on matrices without ties, against the permutation identity
P A = L U, and against numpy.linalg.solve (tests/test_oracle_pivoted.py).
"""
import numpy as np


def gepp(A):
    """Returns (LU, ipiv, info): unit-lower L below the diagonal, U on and
    above, ipiv 1-based row interchanges."""
    LU = np.array(A, dtype=np.float64, copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(n, dtype=np.int64)
    info = 0
    with np.errstate(divide="ignore", invalid="ignore"):
        for k in range(n):
            mag = np.abs(LU[k:, k])
            p = k + int(np.argmax(mag)) if n - k > 0 else k  # first maximum
            if not mag[p - k] > 0.0:
                if mag[p - k] == 0.0 and info == 0:
                    info = k + 1
                p = k
            ipiv[k] = p + 1
            if p != k:
                LU[[k, p], :] = LU[[p, k], :]
            LU[k + 1:, k] /= LU[k, k]
            LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, ipiv, info


def permutation(ipiv):
    """perm[i] = original row that ends in row i after the interchanges."""
    n = len(ipiv)
    perm = np.arange(n)
    for k in range(n):
        p = int(ipiv[k]) - 1
        perm[[k, p]] = perm[[p, k]]
    return perm


def gepp_solve(LU, ipiv, B):
    """X = A^-1 B from the factors of gepp: B permuted, then L, then U."""
    B2 = np.asarray(B, dtype=np.float64)
    vec = B2.ndim == 1
    Y = np.array(B2.reshape(B2.shape[0], -1)[permutation(ipiv)], copy=True)
    n = LU.shape[0]
    for j in range(n):
        Y[j + 1:] -= np.outer(LU[j + 1:, j], Y[j])
    for j in range(n - 1, -1, -1):
        Y[j] /= LU[j, j]
        Y[:j] -= np.outer(LU[:j, j], Y[j])
    return Y[:, 0] if vec else Y
