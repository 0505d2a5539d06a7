"""GPU parity of the adjoint (dA = -A^-T G X^T, dB = A^-T G) with the
oracle's adjoint, a dense FP64 inverse and central finite differences."""
import numpy as np
import pytest
import torch

from oracle import coeffs, solve as osolve
from paper_2312_09376_amd import workloads

pytestmark = pytest.mark.gpu


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


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,k,d", [(1, 1, 2), (5, 2, 2), (129, 1, 2), (300, 3, 1), (1003, 20, 2),
                                   (777, 5, 3)])
def test_backward_matches_oracle(rbt, n, k, d):
    A = workloads.shifted(n, seed=n)
    B = workloads.randn(n, k, seed=1)
    G = workloads.randn(n, k, seed=2)
    _, X, info, _ = rbt.solve_(dev(A), dev(B), d, 2023)
    # solve_ overwrote its A copy with the factors: recompute them
    LU = dev(A)
    rbt.solve_(LU, dev(B), d, 2023)
    dA, dB = rbt.solve_backward(LU, X, dev(G), d, 2023)
    Uo, Vo = coeffs.generate(n, d, 2023)
    Xo, LUo, _ = osolve.rbt_solve(A, B, Uo, Vo, d)
    dAo, dBo = osolve.adjoint(LUo, Xo, G, Uo, Vo, d)
    assert relmax(host(dB), dBo.reshape(n, k)) <= 1e-10
    assert relmax(host(dA), dAo) <= 1e-10


def test_backward_dense_inverse(rbt):
    n, k = 300, 4
    A = workloads.shifted(n, seed=7)
    B = workloads.randn(n, k, seed=8)
    G = workloads.randn(n, k, seed=9)
    X, LU, _, _, _, _ = rbt.solve_refine(dev(A), dev(B), 2, 11)
    dA, dB = rbt.solve_backward(LU, X, dev(G), 2, 11)
    lam = np.linalg.inv(A).T @ G
    Xe = np.linalg.solve(A, B)
    assert relmax(host(dB), lam) <= 1e-11
    assert relmax(host(dA), -lam @ Xe.T) <= 1e-11
    # dA may be skipped
    dA2, dB2 = rbt.solve_backward(LU, X, dev(G), 2, 11, need_dA=False)
    assert dA2 is None and np.array_equal(host(dB2), host(dB))


def test_autograd_gradcheck(rbt):
    torch.manual_seed(0)
    n = 6
    A = (torch.randn(n, n, dtype=torch.float64) / n ** 0.5 + torch.eye(n, dtype=torch.float64)).cuda()
    B = torch.randn(n, 2, dtype=torch.float64).cuda()
    A.requires_grad_(True)
    B.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: rbt.rbt_solve(a, b, 2, 5), (A, B), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)


def test_autograd_finite_differences(rbt):
    """Central differences of L = <C, X> on sampled entries (n = 1024)."""
    n, k = 1024, 8
    A = workloads.shifted(n, seed=21)
    B = workloads.randn(n, k, seed=22)
    C = workloads.randn(n, k, seed=23)
    At = torch.from_numpy(A).cuda().requires_grad_(True)
    Bt = torch.from_numpy(B).cuda().requires_grad_(True)
    Ct = torch.from_numpy(C).cuda()
    X = rbt.rbt_solve(At, Bt, 2, 2023)
    (X * Ct).sum().backward()
    gA, gB = host(At.grad), host(Bt.grad)
    h = 1e-6 * np.abs(A).max()
    rng = np.random.default_rng(0)

    # The difference quotient's noise is the solve error of L over 2h, so the
    # reference solves are refined to the FP64 limit, not just to 10 n eps.
    def loss(Am, Bm):
        X, _, _, _, _, _ = rbt.solve_refine(dev(Am), dev(Bm), 2, 2023, tol=0.0, max_iter=3)
        return float((host(X) * C).sum())

    for _ in range(8):
        i, j = rng.integers(0, n, 2)
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (loss(Ap, B) - loss(Am, B)) / (2 * h)
        assert abs(gA[i, j] - fd) <= 1e-6 * max(1.0, abs(fd))
        c = rng.integers(0, k)
        Bp, Bm = B.copy(), B.copy()
        Bp[i, c] += h
        Bm[i, c] -= h
        fd = (loss(A, Bp) - loss(A, Bm)) / (2 * h)
        assert abs(gB[i, c] - fd) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("n,k,d", [(1, 1, 2), (300, 3, 2), (1003, 8, 2), (513, 20, 1)])
def test_backward_mixed_matches_oracle(rbt, n, k, d):
    """FP32 factors + FP64 refinement of the adjoint solve reach the FP64
    oracle's adjoint to within kappa * 10 n eps."""
    A = workloads.dominant(n, seed=n + 3)
    B = workloads.randn(n, k, seed=1)
    G = workloads.randn(n, k, seed=2)
    X, LU32, _, _, info, _ = rbt.solve_mixed(dev(A), dev(B), d, 2023, prec=rbt.RBT_FP32,
                                             solver=rbt.RBT_IR_GMRES)
    assert int(info.item()) == 0
    dA, dB, iters, berr = rbt.solve_backward_mixed(LU32, dev(A), X, dev(G), d, 2023)
    tol = 10 * n * 2.0 ** -52
    assert float(berr.item()) <= tol
    Uo, Vo = coeffs.generate(n, d, 2023)
    Xo, LUo, _ = osolve.rbt_solve(A, B, Uo, Vo, d)
    dAo, dBo = osolve.adjoint(LUo, Xo, G, Uo, Vo, d)
    kappa = np.linalg.cond(A, np.inf)
    assert relmax(host(dB), dBo.reshape(n, k)) <= 10 * kappa * tol
    assert relmax(host(dA), dAo) <= 10 * kappa * tol
    assert int(iters.item()) <= 6


def test_autograd_mixed_finite_differences(rbt):
    n, k = 512, 4
    A = workloads.shifted(n, seed=31)
    B = workloads.randn(n, k, seed=32)
    C = workloads.randn(n, k, seed=33)
    At = torch.from_numpy(A).cuda().requires_grad_(True)
    Bt = torch.from_numpy(B).cuda().requires_grad_(True)
    X = rbt.rbt_solve(At, Bt, 2, 2023, prec=rbt.RBT_FP32)
    (X * torch.from_numpy(C).cuda()).sum().backward()
    gA, gB = host(At.grad), host(Bt.grad)
    # dense FP64 reference of the same gradient
    lam = np.linalg.solve(A.T, C)
    Xe = np.linalg.solve(A, B)
    assert relmax(gB, lam) <= 1e-9
    assert relmax(gA, -lam @ Xe.T) <= 1e-9


@pytest.mark.parametrize("n,k", [(777, 1), (700, 3), (1000, 8), (600, 16), (500, 20)])
def test_adjoint_residual_backward_error(rbt, n, k):
    """With no refinement the reported backward error is that of the FP32
    adjoint solve (far above the rounding of its FP64 evaluation): it equals
    Eq. 7 of the returned lambda for A^T lambda = G, computed on the host."""
    A = workloads.randn_matrix(n, seed=n + 9)
    B = workloads.randn(n, k, seed=1)
    G = workloads.randn(n, k, seed=2)
    X, LU32, _, _, _, _ = rbt.solve_mixed(dev(A), dev(B), 2, 2023, prec=rbt.RBT_FP32,
                                          solver=rbt.RBT_IR_GMRES)
    _, dB, iters, berr = rbt.solve_backward_mixed(LU32, dev(A), X, dev(G), 2, 2023, max_iter=0,
                                                  need_dA=False)
    assert int(iters.item()) == 0
    lam = host(dB)
    R = G - A.T @ lam
    anorm = np.abs(A).sum(axis=0).max()  # ||A^T||_inf = ||A||_1
    be = max(np.abs(R[:, c]).max() / (anorm * np.abs(lam[:, c]).max() + np.abs(G[:, c]).max())
             for c in range(k))
    assert be > 1e-12  # well above the FP64 rounding of the residual
    assert abs(float(berr.item()) - be) <= 1e-6 * be
