"""Seeded synthetic inputs for RBT solves.

This module is the only code shared by the HIP path's tests/benchmark and the
CPU oracle: it draws matrices and right-hand sides and holds none of the
method's arithmetic (no butterflies, no elimination, no solves).

Matrix families (all square, FP64, column-major when handed to the device):
  randn      i.i.d. N(0,1) entries (the paper's `randn` family, Table 1)
  hostile    randn with the leading 8x8 block scaled by 1e-12: elimination
             without pivoting meets tiny leading pivots unless transformed
  shifted    N(0,1)/sqrt(n) + I (well conditioned, for exact-solution checks)
  orthog     A_ij = sqrt(2/(n+1)) sin(i j pi/(n+1)), symmetric orthogonal
             (Sec. 6.3 failure study), so A^-1 = A
  logcond    Q1 diag(sigma) Q2^T with sigma log-spaced over [1/cond, 1] and
             Haar-distributed orthogonal Q1, Q2: Q of the QR factorization
             of an N(0,1) matrix with the signs of diag(R) made positive
             (Mezzadri, "How to generate random matrices from the classical
             compact groups", 2007)
Host draws use NumPy's PCG64 with the given seed; device draws (large n) use
torch's seeded generator on the GPU.
"""
import math

import numpy as np

MATRIX_SEED = 42   # the paper's tester seeds: matrix 42, right-hand side 64
RHS_SEED = 64
RBT_SEED = 2023


def randn(n, k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal((n, k)))


def randn_matrix(n, seed=MATRIX_SEED):
    return randn(n, n, seed)


def hostile(n, seed=MATRIX_SEED, block=8, scale=1e-12):
    A = randn_matrix(n, seed)
    b = min(block, n)
    A[:b, :b] *= scale
    return A


def shifted(n, seed=MATRIX_SEED):
    A = randn_matrix(n, seed) / math.sqrt(n)
    A[np.diag_indices(n)] += 1.0
    return A


def dominant(n, seed=MATRIX_SEED, scale=0.3):
    """I + scale * N(0,1)/sqrt(n): eigenvalues within about `scale` of 1, so
    the condition number stays O(1) at any n (a matrix every precision of the
    mixed-precision path must refine to full FP64 accuracy)."""
    A = scale * randn_matrix(n, seed) / math.sqrt(n)
    A[np.diag_indices(n)] += 1.0
    return A


def orthog(n):
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.asfortranarray(math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, i) * math.pi / (n + 1)))


def haar_orthogonal(n, seed):
    """Haar-distributed n x n orthogonal matrix: Q R = N(0,1) matrix, then
    each column of Q multiplied by sign(R_jj)."""
    Z = randn_matrix(n, seed)
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def logcond(n, seed=MATRIX_SEED, cond=1e6):
    sigma = np.logspace(0.0, -math.log10(cond), n) if n > 1 else np.ones(1)
    Q1 = haar_orthogonal(n, seed)
    Q2 = haar_orthogonal(n, seed + 1)
    return np.asfortranarray((Q1 * sigma) @ Q2.T)


def batch_sizes(count=2048, lo=37, hi=1500, rhs_lo=1, rhs_hi=16, seed=7):
    """Sizes of a batch of independent systems: n ~ U{lo..hi}, nrhs ~ U{rhs_lo..rhs_hi}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.integers(lo, hi + 1, size=count)
    k = rng.integers(rhs_lo, rhs_hi + 1, size=count)
    return n.astype(np.int64), k.astype(np.int64)


# ---- device-side draws for sizes where host generation would dominate ----

def device_randn(n, k, seed, device="cuda", dtype=None):
    """Column-major (n x k) FP64 N(0,1) tensor drawn on the device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.randn((k, n), generator=g, device=device, dtype=dtype or torch.float64)
    return t.t()   # stride (1, n): column-major view


def device_hostile(n, seed=MATRIX_SEED, block=8, scale=1e-12, device="cuda"):
    A = device_randn(n, n, seed, device)
    b = min(block, n)
    A[:b, :b] *= scale
    return A


def device_haar_orthogonal(n, seed, device="cuda"):
    """As haar_orthogonal, with the N(0,1) matrix drawn and factored on the
    device (QR by the vendor library; input generation only)."""
    import torch
    Z = device_randn(n, n, seed, device)
    Q, R = torch.linalg.qr(Z)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    Q *= d
    del Z, R
    return Q


def device_logcond(n, seed=MATRIX_SEED, cond=1e6, device="cuda"):
    """Column-major Q1 diag(sigma) Q2^T on the device, sigma log-spaced from 1
    to 1/cond, Q1 and Q2 Haar-distributed (device_haar_orthogonal with seeds
    seed and seed + 1)."""
    import torch
    sigma = torch.logspace(0.0, -math.log10(cond), n, dtype=torch.float64, device=device)
    Q1 = device_haar_orthogonal(n, seed, device)
    Q1 *= sigma                              # Q1 diag(sigma)
    Q2 = device_haar_orthogonal(n, seed + 1, device)
    At = Q2 @ Q1.t()                         # (Q1 diag(sigma) Q2^T)^T, row-major
    del Q1, Q2
    return At.t()                            # column-major view of A


def device_shifted(n, seed=MATRIX_SEED, device="cuda"):
    A = device_randn(n, n, seed, device) / math.sqrt(n)
    A.diagonal().add_(1.0)
    return A
