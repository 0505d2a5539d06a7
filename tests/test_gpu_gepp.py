"""GPU parity of the partial-pivoting elimination (the robust re-solve of the
Sec. 5 fallback) against the oracle's GEPP (oracle/pivoted.py), and of the
guarded solvers that fall back to it when the RBT solve cannot be refined:
`orthog` at n = 8192 with a depth-2 RBT (Sec. 6.3, Table 1) and the Eq. 6
family, whose transformed matrix has an exactly zero pivot."""
import numpy as np
import pytest
import torch

from oracle import pivoted, solve as osolve
from paper_2312_09376_amd import workloads

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def rbt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_09376_amd import rbt as r
    r.lib()
    return r


def dev(a):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n", [1, 5, 127, 128, 129, 300, 1003])
def test_gepp_matches_oracle(rbt, n):
    """Same pivots as the oracle (N(0,1) entries: no ties), factors within
    the componentwise bound of two orderings of the same elimination."""
    A = workloads.randn_matrix(n, seed=n + 50)
    LU, ipiv, info = rbt.gepp(dev(A))
    LUo, ipiv_o, info_o = pivoted.gepp(A)
    assert int(info.item()) == info_o == 0
    assert np.array_equal(host(ipiv), ipiv_o)
    den = np.abs(np.tril(LUo, -1) + np.eye(n)) @ np.abs(np.triu(LUo))
    assert (np.abs(host(LU) - LUo) <= 4 * n * EPS * den + 1e-300).all()


@pytest.mark.parametrize("n,k", [(300, 1), (1003, 3), (2000, 20)])
def test_gepp_solve_matches_lapack(rbt, n, k):
    A = workloads.randn_matrix(n, seed=n)
    B = workloads.randn(n, k, seed=5)
    LU, ipiv, _ = rbt.gepp(dev(A))
    X = host(rbt.gepp_solve(LU, ipiv, dev(B)))
    Xl = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A, np.inf)
    assert np.abs(X - Xl).max() <= 10 * kappa * n * EPS * np.abs(Xl).max()
    assert osolve.backward_error(A, X, B) <= 10 * n * EPS


def test_gepp_zero_column_info(rbt):
    n = 200
    A = workloads.randn_matrix(n, seed=1)
    A[:, 130] = 0.0
    _, ipiv, info = rbt.gepp(dev(A))
    _, ipiv_o, info_o = pivoted.gepp(A)
    assert int(info.item()) == info_o == 131
    assert np.array_equal(host(ipiv)[:130], ipiv_o[:130])


def test_guarded_randn_keeps_rbt(rbt):
    n = 1000
    A = workloads.randn_matrix(n)
    B = workloads.randn(n, 1, seed=64)
    X, _, iters, berr, info, path, _ = rbt.solve_guarded(dev(A), dev(B), 2, 2023)
    assert int(path.item()) == 0 and float(berr.item()) <= 10 * n * EPS
    assert osolve.backward_error(A, host(X), B) <= 10 * n * EPS


def test_guarded_orthog_falls_back_to_pivoting(rbt):
    """Sec. 6.3: orthog at n = 8192 defeats the depth-2 RBT even with
    refinement; the guarded solve re-solves with partial pivoting. orthog is
    symmetric orthogonal, so x = A b exactly."""
    n = 8192
    A = workloads.orthog(n)
    B = workloads.randn(n, 1, seed=64)
    tol = 10 * n * EPS
    X, _, iters, berr, info, path, _ = rbt.solve_guarded(dev(A), dev(B), 2, 2023, tol=tol,
                                                         max_iter=10)
    its = host(iters)
    assert int(path.item()) == 2, its
    assert float(berr.item()) <= tol
    assert osolve.backward_error(A, host(X), B) <= tol
    x_exact = A @ B
    assert np.abs(host(X) - x_exact).max() <= 10 * tol * np.abs(x_exact).max()


def test_guarded_eq6_family_falls_back(rbt):
    """A zero pivot of A~ (the Eq. 6 family at depth 2) gives a NaN backward
    error, which ends the RBT refinement at once; the pivoted re-solve is
    exact on this permutation."""
    n = 1000
    A = np.kron(np.eye(n // 2), np.array([[0.0, 1.0], [1.0, 0.0]]))
    B = workloads.randn(n, 2, seed=9)
    X, _, iters, berr, info, path, _ = rbt.solve_guarded(dev(A), dev(B), 2, 2023)
    assert int(path.item()) == 2
    assert host(info)[0] == 1 and host(info)[1] == 0
    assert np.abs(host(X) - A @ B).max() <= 1e-14


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_guarded_orthog_reaches_pivoting(rbt, prec):
    """The mixed solver's fallback chain on orthog at n = 8192: low-precision
    factors, then FP64 RBT factors, then partial pivoting (path 2)."""
    n = 8192
    A = workloads.orthog(n)
    B = workloads.randn(n, 1, seed=64)
    tol = 10 * n * EPS
    p = rbt.RBT_FP32 if prec == "fp32" else rbt.RBT_BF16
    X, _, _, its, berr, info, path, _ = rbt.solve_mixed_guarded(
        dev(A), dev(B), 2, 2023, prec=p, solver=rbt.RBT_IR_GMRES, tol=tol, max_iter=30,
        max_iter64=10)
    assert int(path.item()) == 2, host(its)
    assert float(berr.item()) <= tol
    assert osolve.backward_error(A, host(X), B) <= tol
