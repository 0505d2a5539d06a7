"""Emulated low-precision elimination for the mixed-precision path.
ORACLE: test infrastructure only.

The mixed-precision method (refinement of Sec. 5 with a lower-precision
factorization; the paper cites GMRES-IR/IR in several precisions) keeps A in
FP64, transforms it, rounds A~ to FP32, eliminates without pivoting in FP32
(or with BF16-rounded operands and FP32 accumulation in the trailing update),
and refines the solution in FP64.

The kernels' summation order differs from this emulation, so the factors are
compared entry by entry within a bound derived from the componentwise
backward error of elimination, and the final FP64 solution with the FP64
oracle (error stated per result). Pinned in tests/test_oracle_lowprec.py
(exact dyadic factors, the scalar definition at block width 1, componentwise
backward-error bounds, LAPACK solution). Refinement iteration counts: parity
unpinned.
"""
import numpy as np

from . import transform, solve


def round_bf16(x):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def genp_f32(At, nb=128, bf16_update=False):
    """Blocked elimination in FP32.  With bf16_update the trailing-update
    operands are rounded to BF16 (products accumulated in FP32)."""
    LU = np.array(At, dtype=np.float32, copy=True)
    n = LU.shape[0]
    info = 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for k0 in range(0, n, nb):
            k1 = min(k0 + nb, n)
            for k in range(k0, k1):
                p = LU[k, k]
                if p == 0.0 and info == 0:
                    info = k + 1
                LU[k + 1:, k] /= p
                LU[k + 1:, k + 1:k1] -= np.outer(LU[k + 1:, k], LU[k, k + 1:k1])
            if k1 < n:
                for k in range(k0, k1):
                    LU[k + 1:k1, k1:] -= np.outer(LU[k + 1:k1, k], LU[k, k1:])
                L21 = LU[k1:, k0:k1]
                U12 = LU[k0:k1, k1:]
                if bf16_update:
                    L21, U12 = round_bf16(L21), round_bf16(U12)
                LU[k1:, k1:] -= (L21 @ U12).astype(np.float32)
    return LU, info


def mixed_solve(A, B, U, V, d, tol, max_iter, bf16_update=False):
    """FP32 (or BF16-operand) factorization + FP64 refinement.

    Returns (X, iterations, backward error).
    """
    At = transform.two_sided(A, U, V, d).astype(np.float32)
    LU32, _ = genp_f32(At, bf16_update=bf16_update)
    LU = LU32.astype(np.float64)

    def inner(R):
        Rt = transform.apply_transpose_left(R, U, d).astype(np.float32)
        Y = solve.lu_solve(LU, Rt.astype(np.float64)).astype(np.float32)
        return transform.apply_left(Y.astype(np.float64), V, d)

    X = inner(np.asarray(B, dtype=np.float64))
    it = 0
    be = solve.backward_error(A, X, B)
    while be > tol and it < max_iter:
        X = X + inner(np.asarray(B) - A @ X)
        it += 1
        be = solve.backward_error(A, X, B)
    return X, it, be
