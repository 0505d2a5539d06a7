"""Pins of the oracle's partial-pivoting elimination (oracle/pivoted.py), the
robust re-solve of the Sec. 5 fallback: LAPACK getrf/getrs (scipy), the
identity P A = L U, zero-pivot reporting, and a matrix on which unpivoted
elimination fails."""
import numpy as np
import pytest
import scipy.linalg

from oracle import pivoted, solve
from paper_2312_09376_amd import workloads


@pytest.mark.parametrize("n", [1, 2, 5, 31, 128, 200])
def test_gepp_matches_lapack_getrf(n):
    A = workloads.randn_matrix(n, seed=n + 3)
    LU, ipiv, info = pivoted.gepp(A)
    lu_l, piv_l = scipy.linalg.lu_factor(A)
    assert info == 0
    assert np.array_equal(ipiv, piv_l + 1)  # scipy's pivots are 0-based
    assert np.allclose(LU, lu_l, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("n", [3, 64, 257])
def test_gepp_permutation_identity(n):
    A = workloads.randn_matrix(n, seed=7 * n)
    LU, ipiv, _ = pivoted.gepp(A)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    P = pivoted.permutation(ipiv)
    assert sorted(P.tolist()) == list(range(n))
    assert np.abs(A[P] - L @ U).max() <= 8 * n * 2.0 ** -52 * (np.abs(L) @ np.abs(U)).max()
    assert np.abs(L).max() <= 1.0  # partial pivoting bounds the multipliers


def test_gepp_solve_matches_lapack():
    n = 150
    A = workloads.randn_matrix(n, seed=11)
    B = workloads.randn(n, 3, seed=12)
    LU, ipiv, _ = pivoted.gepp(A)
    X = pivoted.gepp_solve(LU, ipiv, B)
    Xl = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), B)
    assert np.allclose(X, Xl, rtol=1e-11, atol=1e-12)
    assert solve.backward_error(A, X, B) <= 10 * n * 2.0 ** -52


def test_gepp_zero_pivot_and_unpivoted_failure():
    A = np.array([[0.0, 1.0, 2.0], [0.0, 3.0, 4.0], [0.0, 5.0, 7.0]])
    _, ipiv, info = pivoted.gepp(A)
    assert info == 1 and ipiv[0] == 1  # zero column: recorded, not interchanged
    # the Eq. 6 matrix: unpivoted elimination meets a zero pivot, GEPP does not
    P = np.kron(np.eye(2), np.array([[0.0, 1.0], [1.0, 0.0]]))
    _, info_np = solve.genp_unblocked(P)
    LU, ipiv, info = pivoted.gepp(P)
    assert info_np == 1 and info == 0
    assert np.allclose(pivoted.gepp_solve(LU, ipiv, np.arange(4.0)), P @ np.arange(4.0))
