"""GPU parity of the mixed-precision path (FP32 or BF16-update elimination of
A~ = U^T A V, FP64 refinement with the original A) against the FP64 oracle.

The low-precision factors are compared with the oracle's emulation
(oracle/lowprec.py) entry by entry, within a bound derived from the
componentwise backward error of elimination (factor_tolerance); the final
FP64 solution is compared with the FP64 oracle solution, and the backward
error with the refinement tolerance."""
import numpy as np
import pytest
import torch

from oracle import coeffs, lowprec, solve as osolve, transform as otr
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


def relfro(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,k,d", [(1, 1, 2), (5, 2, 2), (129, 1, 2), (300, 3, 1), (1003, 2, 2),
                                   (777, 20, 3), (513, 1, 0)])
def test_mixed_converges_to_oracle_solution(rbt, prec, n, k, d):
    A = workloads.dominant(n, seed=n + 1)
    B = workloads.randn(n, k, seed=3)
    p = rbt.RBT_FP32 if prec == "fp32" else rbt.RBT_BF16
    tol = 10 * n * EPS
    X, LU, iters, berr, info, _ = rbt.solve_mixed(dev(A), dev(B), d, 2023, prec=p, tol=tol,
                                                  max_iter=40)
    assert int(info.item()) == 0
    be = float(berr.item())
    assert be <= tol, (be, int(iters.item()))
    Uo, Vo = coeffs.generate(n, d, 2023)
    Xo, _, _ = osolve.rbt_solve(A, B, Uo, Vo, d)
    # both solutions are within kappa * (backward error) of A^-1 B
    kappa = np.linalg.cond(A, np.inf)
    assert relfro(host(X), Xo) <= 10 * kappa * tol
    it = int(iters.item())
    assert it <= (4 if prec == "fp32" else 12), it


def factor_tolerance(LUo, bf16):
    """Element-wise bound for two computations of the same low-precision
    elimination that differ only in the order of their FP32 roundings
    (blocking, summation order of the matrix products): each side's factors
    reproduce A~ with componentwise error <= gamma_n |L| |U| (Higham, Thm.
    9.3), so on matrices with well-conditioned leading minors an entry of the
    two factor sets differs by at most a few n u32 (|L| |U|)_ij. With BF16
    operands both sides round the same FP32 operands to BF16, but an operand
    that differs by an FP32 rounding can round to the neighbouring BF16 value:
    each product of a sum then moves by at most 2 * 2^-7 of its size, which
    adds 2^-6 (|L| |U|)_ij."""
    LU = LUo.astype(np.float64)
    n = LU.shape[0]
    den = np.abs(np.tril(LU, -1) + np.eye(n)) @ np.abs(np.triu(LU))
    tol = 4 * n * 2.0 ** -24 * den
    if bf16:
        tol += 2.0 ** -6 * den
    return tol


def assert_factors_match(LUg, LUo, bf16):
    tol = factor_tolerance(LUo, bf16)
    diff = np.abs(LUg.astype(np.float64) - LUo.astype(np.float64))
    bad = np.argwhere(diff > tol)
    assert bad.size == 0, (len(bad), bad[:5].tolist(), float((diff / tol).max()))
    return float((diff / np.where(tol > 0, tol, 1.0)).max())


def test_mixed_fp32_factors_match_emulation(rbt):
    n, d = 300, 2
    A = workloads.dominant(n, seed=5)
    B = workloads.randn(n, 1, seed=6)
    _, LU, _, _, info, _ = rbt.solve_mixed(dev(A), dev(B), d, 2023, prec=rbt.RBT_FP32)
    Uo, Vo = coeffs.generate(n, d, 2023)
    At = otr.two_sided(A, Uo, Vo, d).astype(np.float32)
    LUo, info_o = lowprec.genp_f32(At)
    assert int(info.item()) == info_o == 0
    assert_factors_match(host(LU), LUo, bf16=False)


def test_mixed_bf16_uses_bf16_operands(rbt):
    """BF16 factors agree with the BF16 emulation element by element, and
    are not the FP32 factors (the operands really are rounded)."""
    n, d = 600, 2
    A = workloads.dominant(n, seed=8)
    B = workloads.randn(n, 1, seed=9)
    _, LU32, _, _, _, _ = rbt.solve_mixed(dev(A), dev(B), d, 2023, prec=rbt.RBT_FP32)
    _, LU16, _, _, _, _ = rbt.solve_mixed(dev(A), dev(B), d, 2023, prec=rbt.RBT_BF16)
    a32 = host(LU32)
    a16 = host(LU16)
    Uo, Vo = coeffs.generate(n, d, 2023)
    At = otr.two_sided(A, Uo, Vo, d).astype(np.float32)
    LUe, _ = lowprec.genp_f32(At, bf16_update=True)
    assert_factors_match(a16, LUe, bf16=True)
    LU32e, _ = lowprec.genp_f32(At)
    assert_factors_match(a32, LU32e, bf16=False)
    # far outside the FP32 bound somewhere: BF16 rounding took place
    assert (np.abs(a16.astype(np.float64) - a32) > factor_tolerance(LU32e, bf16=False)).any()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [1536, 2500])
def test_mixed_factors_elementwise_multi_panel(rbt, prec, n):
    """Panels of W = 512 < n: every trailing update runs the FP32 trailing
    GEMM (k_sgemm, trailing instance) or, with BF16 updates, the staged BF16
    GEMM (k_hgemm), and the panel steps run the depth-128 updates; the
    factors are compared with the emulation entry by entry (n = 2500 also
    leaves a ragged last block of 68 rows)."""
    from paper_2312_09376_amd import _lib
    d = 2
    bf16 = prec == "bf16"
    A = workloads.dominant(n, seed=n)
    B = workloads.randn(n, 1, seed=2)
    old = rbt.get_option(_lib.RBT_OPT_OUTER_NB)
    try:
        rbt.set_option(_lib.RBT_OPT_OUTER_NB, 512)
        _, LU, _, _, info, _ = rbt.solve_mixed(
            dev(A), dev(B), d, 2023, prec=rbt.RBT_BF16 if bf16 else rbt.RBT_FP32, max_iter=0)
        LUg = host(LU)
    finally:
        rbt.set_option(_lib.RBT_OPT_OUTER_NB, old)
    Uo, Vo = coeffs.generate(n, d, 2023)
    At = otr.two_sided(A, Uo, Vo, d).astype(np.float32)
    LUo, info_o = lowprec.genp_f32(At, bf16_update=bf16)
    assert int(info.item()) == info_o == 0
    worst = assert_factors_match(LUg, LUo, bf16)
    print(f"n={n} {prec}: worst |diff| / bound = {worst:.3g}")


def test_mixed_fp32_randn_refines_to_tolerance(rbt):
    n = 512
    A = workloads.randn_matrix(n, seed=42)
    B = workloads.randn(n, 1, seed=64)
    tol = 10 * n * EPS
    X, _, iters, berr, info, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_FP32,
                                                 tol=tol, max_iter=40)
    assert int(info.item()) == 0
    assert float(berr.item()) <= tol
    Xe = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A, np.inf)
    assert relfro(host(X), Xe) <= 20 * kappa * tol


def test_mixed_zero_pivot_reports_info(rbt):
    A = np.eye(200)
    A[130, 130] = 0.0
    A[130, 131] = 1.0
    A[131, 130] = 1.0
    B = np.ones((200, 1))
    _, _, iters, berr, info, _ = rbt.solve_mixed(dev(A), dev(B), 0, 1, prec=rbt.RBT_FP32,
                                                 max_iter=3)
    assert int(info.item()) == 131
    assert not (float(berr.item()) <= 1.0)  # NaN/Inf never looks converged
    assert int(iters.item()) == 3


def test_mixed_empty(rbt):
    A = torch.empty_strided((0, 0), (1, 1), dtype=torch.float64, device="cuda")
    B = torch.empty_strided((0, 1), (1, 1), dtype=torch.float64, device="cuda")
    X, _, iters, berr, info, _ = rbt.solve_mixed(A, B, 2, 1)
    assert int(iters.item()) == 0 and float(berr.item()) == 0.0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,k,d", [(1, 1, 2), (300, 3, 1), (1003, 2, 2), (700, 20, 2)])
def test_gmres_ir_converges_to_oracle_solution(rbt, prec, n, k, d):
    A = workloads.dominant(n, seed=n + 7)
    B = workloads.randn(n, k, seed=4)
    p = rbt.RBT_FP32 if prec == "fp32" else rbt.RBT_BF16
    tol = 10 * n * EPS
    X, _, iters, berr, info, _ = rbt.solve_mixed(dev(A), dev(B), d, 2023, prec=p,
                                                 solver=rbt.RBT_IR_GMRES, tol=tol, max_iter=60)
    assert int(info.item()) == 0
    assert float(berr.item()) <= tol
    Uo, Vo = coeffs.generate(n, d, 2023)
    Xo, _, _ = osolve.rbt_solve(A, B, Uo, Vo, d)
    kappa = np.linalg.cond(A, np.inf)
    assert relfro(host(X), Xo) <= 10 * kappa * tol
    assert int(iters.item()) <= (8 if prec == "fp32" else 20)


def test_gmres_ir_fp32_randn_beats_classical(rbt):
    """N(0,1) at n = 1536: GMRES-IR reaches the tolerance in fewer Krylov
    iterations than classical refinement needs corrections."""
    n = 1536
    A = workloads.randn_matrix(n, seed=42)
    B = workloads.randn(n, 1, seed=64)
    tol = 10 * n * EPS
    Xg, _, itg, beg, _, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_FP32,
                                            solver=rbt.RBT_IR_GMRES, tol=tol, max_iter=100)
    Xc, _, itc, bec, _, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_FP32,
                                            solver=rbt.RBT_IR_CLASSIC, tol=tol, max_iter=100)
    assert float(beg.item()) <= tol
    assert int(itg.item()) < int(itc.item()) or float(bec.item()) > tol
    Xe = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A, np.inf)
    assert relfro(host(Xg), Xe) <= 20 * kappa * tol


def test_gmres_ir_respects_iteration_cap(rbt):
    n = 512
    A = workloads.randn_matrix(n, seed=42)
    B = workloads.randn(n, 2, seed=64)
    _, _, iters, berr, _, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_BF16,
                                              solver=rbt.RBT_IR_GMRES, tol=0.0, max_iter=7)
    assert int(iters.item()) == 7
    assert np.isfinite(float(berr.item()))


def test_guarded_without_fallback_matches_mixed(rbt):
    """When the low-precision factors reach tol, the guarded solve is the
    mixed solve: same result bit for bit, no FP64 factorization."""
    n = 700
    A = workloads.dominant(n, seed=21)
    B = workloads.randn(n, 3, seed=22)
    Xm, _, itm, bem, _, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_FP32,
                                            solver=rbt.RBT_IR_GMRES, max_iter=30)
    Xg, _, _, its, beg, info, path, _ = rbt.solve_mixed_guarded(dev(A), dev(B), 2, 2023,
                                                                prec=rbt.RBT_FP32,
                                                                solver=rbt.RBT_IR_GMRES,
                                                                max_iter=30)
    assert int(path.item()) == 0
    assert host(its).tolist() == [int(itm.item()), 0]
    assert host(info).tolist() == [0, 0]
    assert np.array_equal(host(Xg), host(Xm))
    assert float(beg.item()) == float(bem.item()) <= 10 * n * EPS


@pytest.mark.parametrize("n,k", [(700, 1), (333, 5)])
def test_guarded_fallback_matches_fp64_oracle(rbt, n, k):
    """BF16 factors of an N(0,1) matrix with no refinement budget cannot
    reach 10 n eps, so the FP64 factors of the same A~ are computed: they
    reconstruct the oracle's A~ to FP64 accuracy (elementwise agreement of
    unpivoted factors of an N(0,1) matrix has no fixed tolerance), and the
    refined solution reaches the tolerance."""
    A = workloads.randn_matrix(n, seed=n)
    B = workloads.randn(n, k, seed=5)
    tol = 10 * n * EPS
    X, _, LU64, its, berr, info, path, _ = rbt.solve_mixed_guarded(
        dev(A), dev(B), 2, 2023, prec=rbt.RBT_BF16, solver=rbt.RBT_IR_CLASSIC, tol=tol,
        max_iter=0, max_iter64=10)
    assert int(path.item()) == 1
    assert host(info).tolist() == [0, 0]
    assert host(its)[0] == 0
    assert float(berr.item()) <= tol
    Uo, Vo = coeffs.generate(n, 2, 2023)
    At = otr.two_sided(A, Uo, Vo, 2)
    F = host(LU64)
    Lm = np.tril(F, -1) + np.eye(n)
    Um = np.triu(F)
    assert np.abs(Lm @ Um - At).max() / (np.abs(Lm).max() * np.abs(Um).max()) <= 20 * n * EPS
    Xe = np.linalg.solve(A, B)
    assert relfro(host(X), Xe) <= 20 * np.linalg.cond(A, np.inf) * tol


def test_guarded_gmres_stall_rule(rbt):
    """tol = 0 is out of reach of any extrapolation, so the GMRES phase stops
    after the minimum of 8 iterations of its first cycle (unless the cycle
    ended before), the FP64 RBT phase cannot reach it either, and the
    pivoted re-solve (path 2) spends its whole budget."""
    n = 400
    A = workloads.randn_matrix(n, seed=77)
    B = workloads.randn(n, 2, seed=78)
    X, _, _, its, berr, info, path, _ = rbt.solve_mixed_guarded(
        dev(A), dev(B), 2, 2023, prec=rbt.RBT_BF16, solver=rbt.RBT_IR_GMRES, tol=0.0,
        max_iter=100, max_iter64=2)
    its = host(its)
    assert int(path.item()) == 2
    assert 1 <= its[0] <= 8 and its[1] == 2
    assert float(berr.item()) <= 10 * n * EPS
    assert relfro(host(X), np.linalg.solve(A, B)) <= 20 * np.linalg.cond(A, np.inf) * 10 * n * EPS


def test_guarded_classic_stall_rule(rbt):
    """Classical refinement with BF16 factors of an N(0,1) matrix stops at the
    first correction that does not halve the backward error, long before the
    budget, and the FP64 fallback reaches the tolerance."""
    n = 900
    A = workloads.randn_matrix(n, seed=9)
    B = workloads.randn(n, 1, seed=10)
    _, _, _, its, berr, _, path, _ = rbt.solve_mixed_guarded(
        dev(A), dev(B), 2, 2023, prec=rbt.RBT_BF16, solver=rbt.RBT_IR_CLASSIC, max_iter=200)
    its = host(its)
    if int(path.item()) == 1:
        assert its[0] < 200
    assert float(berr.item()) <= 10 * n * EPS


@pytest.mark.parametrize("n,W", [(3000, 1024), (1003, 256), (700, 128), (2500, 512)])
def test_bf16_staged_gemm_identical(rbt, n, W):
    """The staged BF16 trailing GEMM (operands rounded once, 256 x 256
    tiles) sums the same BF16 products in the same order as the
    tile-by-tile path: the factors are bit-identical."""
    A = workloads.dominant(n, seed=n + 2)
    B = workloads.randn(n, 1, seed=1)
    old_w = rbt.get_option(rbt._lib.RBT_OPT_OUTER_NB)
    rbt.set_option(rbt._lib.RBT_OPT_OUTER_NB, W)
    try:
        out = {}
        for staged in (0, 1):
            rbt.set_option(rbt._lib.RBT_OPT_BF16_STAGED, staged)
            X, LU, _, _, _, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_BF16,
                                                max_iter=2)
            torch.cuda.synchronize()
            out[staged] = (host(LU), host(X))
        assert np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][1], out[1][1])
    finally:
        rbt.set_option(rbt._lib.RBT_OPT_BF16_STAGED, 1)
        rbt.set_option(rbt._lib.RBT_OPT_OUTER_NB, old_w)
