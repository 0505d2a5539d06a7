"""Pins of the oracle's elimination, solves, backward error, refinement and
adjoint (Eq. 1, Eq. 5, Eq. 7, Sec. 5)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import coeffs, lowprec, solve, transform
from paper_2312_09376_amd import workloads


def _gen(n, d, seed=2023):
    return coeffs.generate(n, d, seed)


def test_lu_reconstruction():
    for n in (1, 2, 3, 17, 64, 150):
        A = workloads.randn_matrix(n, seed=n)
        LU, info = solve.genp_unblocked(A)
        assert info == 0
        L = np.tril(LU, -1) + np.eye(n)
        Uf = np.triu(LU)
        err = np.abs(L @ Uf - A).max() / (np.abs(L).max() * np.abs(Uf).max() * n)
        assert err < 4 * n * 2.0 ** -53


def test_lu_matches_exact_rational_elimination():
    """Tiny n: the float factors equal the exact rational ones to rounding."""
    rng = np.random.default_rng(1)
    n = 7
    A = rng.integers(-5, 6, (n, n)).astype(float) + 12 * np.eye(n)
    M = [[Fraction(int(v)) for v in row] for row in A]
    for k in range(n):
        for i in range(k + 1, n):
            M[i][k] = M[i][k] / M[k][k]
            for j in range(k + 1, n):
                M[i][j] -= M[i][k] * M[k][j]
    exact = np.array([[float(v) for v in row] for row in M])
    LU, _ = solve.genp_unblocked(A)
    assert np.allclose(LU, exact, rtol=1e-14, atol=1e-14)


def test_blocked_equals_unblocked():
    A = workloads.randn_matrix(300, seed=3) + 30 * np.eye(300)
    a, _ = solve.genp_unblocked(A)
    b, _ = solve.genp_blocked(A, nb=64)
    c, _ = solve.genp_blocked(A, nb=37)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    assert np.allclose(a, c, rtol=1e-12, atol=1e-12)


def test_zero_pivot_info():
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 1.0], [1.0, 1.0, 1.0]])
    _, info = solve.genp_unblocked(A)
    assert info == 2
    _, info = solve.genp_blocked(A, nb=2)
    assert info == 2


def test_triangular_solves_against_library():
    rng = np.random.default_rng(4)
    n = 60
    LU = rng.standard_normal((n, n)) + 8 * np.eye(n)
    B = rng.standard_normal((n, 3))
    L = np.tril(LU, -1) + np.eye(n)
    Uf = np.triu(LU)
    assert np.allclose(solve.forward_unit_lower(LU, B), np.linalg.solve(L, B))
    assert np.allclose(solve.backward_upper(LU, B), np.linalg.solve(Uf, B))
    assert np.allclose(solve.forward_upper_transposed(LU, B), np.linalg.solve(Uf.T, B))
    assert np.allclose(solve.backward_unit_lower_transposed(LU, B), np.linalg.solve(L.T, B))


@pytest.mark.parametrize("n,d", [(1, 2), (2, 2), (3, 1), (5, 2), (9, 2), (12, 2), (13, 3), (16, 4)])
def test_solution_matches_exact_rational_solve(n, d):
    """n <= 16: the oracle's RBT solve agrees with the exact solution of the
    FP64 inputs (rational elimination) to conditioning-bounded accuracy, and
    with LAPACK's partial-pivoting solve."""
    A = workloads.shifted(n, seed=n)
    b = workloads.randn(n, 1, seed=n + 1)[:, 0]
    U, V = _gen(n, d)
    x, _, info = solve.rbt_solve(A, b, U, V, d)
    assert info == 0
    M = [[Fraction(float(v)) for v in row] + [Fraction(float(bi))] for row, bi in zip(A, b)]
    for k in range(n):
        p = max(range(k, n), key=lambda i: abs(M[i][k]))
        M[k], M[p] = M[p], M[k]
        for i in range(n):
            if i != k:
                f = M[i][k] / M[k][k]
                M[i] = [M[i][j] - f * M[k][j] for j in range(n + 1)]
    exact = np.array([float(M[i][n] / M[i][i]) for i in range(n)])
    kappa = np.linalg.cond(A)
    assert np.abs(x - exact).max() / np.abs(exact).max() < 50 * kappa * 2.0 ** -53
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-13)


def test_solution_randn_moderate():
    n, d = 200, 2
    A = workloads.randn_matrix(n)
    B = workloads.randn(n, 4, seed=64)
    U, V = _gen(n, d)
    X, LU, info = solve.rbt_solve(A, B, U, V, d)
    assert info == 0
    assert solve.backward_error(A, X, B) < 10 * n * 2.0 ** -52
    assert np.allclose(X, np.linalg.solve(A, B), rtol=1e-8, atol=1e-9)


def test_transform_rescues_hostile_matrix():
    """Without the transform the tiny leading block wrecks elimination without
    pivoting; with it the backward error is small."""
    n = 120
    A = workloads.hostile(n)
    b = workloads.randn(n, 1, seed=64)
    U, V = _gen(n, 2)
    X0, _, _ = solve.rbt_solve(A, b, U[:, :0], V[:, :0], 0)
    X2, _, _ = solve.rbt_solve(A, b, U, V, 2)
    assert solve.backward_error(A, X0, b) > 1e-8
    assert solve.backward_error(A, X2, b) < 10 * n * 2.0 ** -52


def test_backward_error_closed_forms():
    """Eq. 7 on cases with a known value, including orthog (A^-1 = A)."""
    n = 50
    b = workloads.randn(n, 1, seed=5)[:, 0]
    x = b.copy()
    x[3] += 1e-3
    expect = 1e-3 / (1.0 * np.abs(x).max() + np.abs(b).max())
    assert math.isclose(solve.backward_error(np.eye(n), x, b), expect, rel_tol=1e-12)
    A = workloads.orthog(n)
    assert np.allclose(A @ A, np.eye(n), atol=1e-13)
    assert solve.backward_error(A, A @ b, b) < 4 * n * 2.0 ** -53
    # two columns: the maximum over columns
    B = np.stack([b, b], axis=1)
    X = np.stack([b, x], axis=1)
    assert math.isclose(solve.backward_error(np.eye(n), X, B), expect, rel_tol=1e-12)


def test_orthog_solution_closed_form():
    """orthog: x = A b exactly; the RBT solve reaches it to rounding times the
    growth the transform leaves (small at this size)."""
    n = 64
    A = workloads.orthog(n)
    b = workloads.randn(n, 1, seed=2)[:, 0]
    U, V = _gen(n, 2)
    x, _, _ = solve.rbt_solve(A, b, U, V, 2)
    assert np.abs(x - A @ b).max() < 1e-8


def test_growth_bound_eq5():
    """Eq. 5: every Schur-complement entry after k elimination steps is at most
    sqrt(n) ||A~||_2 / sigma_k(A~[:k,:k]) * max|A~|."""
    n = 40
    A = workloads.randn_matrix(n, seed=8)
    U, V = _gen(n, 2)
    At = transform.two_sided(A, U, V, 2)
    S = At.copy()
    norm2 = np.linalg.norm(At, 2)
    amax = np.abs(At).max()
    for k in range(1, n):
        p = S[k - 1, k - 1]
        S[k:, k - 1] /= p
        S[k:, k:] -= np.outer(S[k:, k - 1], S[k - 1, k:])
        sk = np.linalg.svd(At[:k, :k], compute_uv=False).min()
        bound = math.sqrt(n) * norm2 / sk * amax
        assert np.abs(S[k:, k:]).max() <= bound * (1 + 1e-10)
    LU, _ = solve.genp_unblocked(At)
    assert np.allclose(np.triu(LU), np.triu(S), rtol=1e-12, atol=1e-12)


def test_refinement_converges():
    n = 150
    A = workloads.randn_matrix(n, seed=4)
    B = workloads.randn(n, 2, seed=64)
    U, V = _gen(n, 2)
    X, LU, _ = solve.rbt_solve(A, B, U, V, 2)
    tol = 1e-15
    X2, it, be = solve.refine(A, B, X, LU, U, V, 2, tol=tol, max_iter=5)
    assert be <= max(tol, 4 * 2.0 ** -53) or it == 5
    assert be <= solve.backward_error(A, X, B)


def test_adjoint_dense_inverse_and_finite_differences():
    n, k, d = 24, 3, 2
    A = workloads.shifted(n, seed=3)
    B = workloads.randn(n, k, seed=4)
    C = workloads.randn(n, k, seed=5)       # loss = <C, X>
    U, V = _gen(n, d)
    X, LU, _ = solve.rbt_solve(A, B, U, V, d)
    dA, dB = solve.adjoint(LU, X, C, U, V, d)
    Ainv = np.linalg.inv(A)
    lam = Ainv.T @ C
    assert np.allclose(dB, lam, rtol=1e-10, atol=1e-12)
    assert np.allclose(dA, -lam @ X.T, rtol=1e-10, atol=1e-12)
    h = 1e-6 * np.abs(A).max()
    rng = np.random.default_rng(0)
    for _ in range(12):
        i, j = rng.integers(0, n, 2)
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (np.sum(C * np.linalg.solve(Ap, B)) - np.sum(C * np.linalg.solve(Am, B))) / (2 * h)
        assert math.isclose(dA[i, j], fd, rel_tol=1e-6, abs_tol=1e-8)
        c = rng.integers(0, k)
        Bp, Bm = B.copy(), B.copy()
        Bp[i, c] += h
        Bm[i, c] -= h
        fd = (np.sum(C * np.linalg.solve(A, Bp)) - np.sum(C * np.linalg.solve(A, Bm))) / (2 * h)
        assert math.isclose(dB[i, c], fd, rel_tol=1e-6, abs_tol=1e-8)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32),
                        np.float32([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(lowprec.round_bf16(x), ref)


def test_mixed_precision_emulation_refines_to_fp64():
    n = 200
    A = workloads.randn_matrix(n, seed=6)
    B = workloads.randn(n, 1, seed=64)
    U, V = _gen(n, 2)
    tol = 10 * n * 2.0 ** -52
    X, it, be = lowprec.mixed_solve(A, B, U, V, 2, tol, 30)
    assert be <= tol and it >= 1
    # BF16 operands with classical refinement: converges when kappa * 2^-8 is
    # small (shifted matrix), does not on randn at kappa ~ 1e3.
    As = workloads.shifted(n, seed=6)
    Xb, itb, beb = lowprec.mixed_solve(As, B, U, V, 2, tol, 100, bf16_update=True)
    assert beb <= tol and itb >= 1
    with np.errstate(all="ignore"):
        _, itn, ben = lowprec.mixed_solve(A, B, U, V, 2, tol, 40, bf16_update=True)
    assert itn == 40 and not ben <= tol
