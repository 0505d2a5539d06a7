"""Pins of the emulated low-precision elimination (oracle/lowprec.py) that
the FP32 / BF16-update factor tests compare the GPU with.

The mixed-precision method keeps the elimination of Sec. 1 (GENP on A~) but
performs it in FP32, or with BF16-rounded operands in the matrix-product
updates; accuracy is recovered by FP64 refinement (Sec. 5). The emulation is
pinned by:
  * exact arithmetic: on an A = L U whose every intermediate value is a short
    dyadic rational, FP32 and BF16-operand elimination are exact and return
    the FP64 factors bit for bit;
  * the definition of elimination written as a scalar FP32 loop (one
    rounding per multiply and per subtract), which the blocked routine must
    reproduce bit for bit when its block width is 1, with and without BF16
    operand rounding (round_bf16 itself is pinned against torch's bfloat16);
  * componentwise backward-error bounds |A - L U| <= c n u |L| |U| (Higham,
    Thm. 9.3) with u = 2^-24 for FP32, and a bound at the BF16 unit
    roundoff 2^-8 for BF16 operands, which the FP32 bound must not cover
    (the rounding really happens);
  * mixed_solve reaching the LAPACK solution within kappa * tol.
"""
import numpy as np
import pytest

from oracle import coeffs, lowprec, solve
from paper_2312_09376_amd import workloads

U32 = 2.0 ** -24
U16 = 2.0 ** -8


def _dyadic_lu(n, seed):
    """Unit-lower L with entries in {0, +-1/2, +-1/4} and upper U with
    diagonal +-1, +-2 and small integer entries: every step of elimination
    on A = L U is exact in FP32 (and every L, U entry is a BF16 value)."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.choice([0.0, 0.5, -0.5, 0.25, -0.25], size=(n, n)), -1) + np.eye(n)
    Uf = np.triu(rng.integers(-3, 4, size=(n, n)).astype(float), 1)
    Uf += np.diag(rng.choice([1.0, -1.0, 2.0, -2.0], size=n))
    return L, Uf


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("n,nb", [(12, 4), (20, 7), (16, 128)])
def test_genp_f32_exact_on_dyadic_factors(n, nb, bf16):
    L, Uf = _dyadic_lu(n, seed=n + nb)
    A = L @ Uf
    # the products stay far below 2^24: FP32 holds A and every Schur
    # complement exactly
    assert np.abs(A).max() < 2.0 ** 12
    expect = np.tril(L, -1) + Uf
    LU32, info = lowprec.genp_f32(A.astype(np.float32), nb=nb, bf16_update=bf16)
    assert info == 0
    assert np.array_equal(LU32.astype(np.float64), expect)
    LU64, _ = solve.genp_unblocked(A)
    assert np.array_equal(LU64, expect)


def _scalar_genp_f32(A, bf16):
    """Elimination without pivoting from its definition, one FP32 rounding per
    operation: l_ik = a_ik / a_kk; a_ij -= l_ik * a_kj (with bf16, both
    factors of the product rounded to BF16 first)."""
    M = [[np.float32(v) for v in row] for row in np.asarray(A, dtype=np.float32)]
    n = len(M)
    rb = (lambda x: np.float32(lowprec.round_bf16(np.float32(x)))) if bf16 else (lambda x: x)
    for k in range(n):
        for i in range(k + 1, n):
            M[i][k] = np.float32(M[i][k] / M[k][k])
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = np.float32(M[i][j] - np.float32(rb(M[i][k]) * rb(M[k][j])))
    return np.array(M, dtype=np.float32)


@pytest.mark.parametrize("bf16", [False, True])
def test_genp_f32_unit_blocks_match_scalar_definition(bf16):
    n = 24
    A = workloads.dominant(n, seed=4)
    ref = _scalar_genp_f32(A, bf16)
    got, _ = lowprec.genp_f32(A.astype(np.float32), nb=1, bf16_update=bf16)
    assert np.array_equal(got, ref)


def _recon_ratio(A32, LU32):
    """max_ij |A - L U|_ij / (|L| |U|)_ij, computed in FP64 from the
    FP32 factors."""
    LU = LU32.astype(np.float64)
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    Uf = np.triu(LU)
    err = np.abs(A32.astype(np.float64) - L @ Uf)
    den = np.abs(L) @ np.abs(Uf)
    return (err / np.where(den > 0, den, 1.0)).max()


def test_genp_f32_componentwise_backward_error():
    n = 300
    A = workloads.dominant(n, seed=11)
    A32 = A.astype(np.float32)
    LU32, info = lowprec.genp_f32(A32, nb=128)
    assert info == 0
    r32 = _recon_ratio(A32, LU32)
    assert r32 <= n * U32, r32  # gamma_n, with rounding to nearest
    LUb, _ = lowprec.genp_f32(A32, nb=128, bf16_update=True)
    rb = _recon_ratio(A32, LUb)
    # one BF16 rounding per operand of each product: relative error of a
    # product <= 2 u16 + u16^2, plus the FP32 accumulation
    assert rb <= (2 * U16 + U16 ** 2) + n * U32, rb
    assert rb > n * U32  # the operands were rounded: not an FP32 result
    # nb = 64 and nb = 128 differ only in rounding order
    LU64b, _ = lowprec.genp_f32(A32, nb=64)
    assert _recon_ratio(A32, LU64b) <= n * U32


def test_genp_f32_zero_pivot_info():
    A = np.eye(10, dtype=np.float32)
    A[6, 6] = 0.0
    A[6, 7] = A[7, 6] = 1.0
    _, info = lowprec.genp_f32(A, nb=4)
    assert info == 7
    _, info64 = solve.genp_unblocked(A.astype(np.float64))
    assert info64 == 7


@pytest.mark.parametrize("bf16", [False, True])
def test_mixed_solve_reaches_lapack_solution(bf16):
    n = 160
    A = workloads.dominant(n, seed=21)
    B = workloads.randn(n, 2, seed=64)
    U, V = coeffs.generate(n, 2, 2023)
    tol = 10 * n * 2.0 ** -52
    X, it, be = lowprec.mixed_solve(A, B, U, V, 2, tol, 50, bf16_update=bf16)
    assert be <= tol and it >= 1
    Xl = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A, np.inf)
    assert np.abs(X - Xl).max() / np.abs(Xl).max() <= 10 * kappa * tol
