"""Butterfly factors and their application.  ORACLE: test infrastructure only.

Convention (Eq. 1, Eq. 3): U = O_d R_d ... O_1 R_1 with R_l = diag(U[:, l-1])
and O_l the block-diagonal of the layer-l butterflies of Eq. 2.  Hence

  U^T x : for l = d, ..., 1: mix with O_l, then scale by U[:, l-1]
  U   x : for l = 1, ..., d: scale by U[:, l-1], then mix with O_l

and the same with V.  Mixing a pair (a, b) (a in the top half) gives
((x_a + x_b)/sqrt2, (x_a - x_b)/sqrt2); an unpaired row is left as is (Eq. 2).
Reading: Algorithm 1's RBT2 scales its inputs before mixing; only
the Eq. 3 order above reproduces the worked example of Eq. 6, so the oracle
follows Eq. 3.

Parity: the dense factors are pinned by the Eq. 6 example, orthogonality,
the Sylvester-Hadamard special case (scipy.linalg.hadamard) and the Parker
recursion; the packed routines are pinned by equality with the dense products.
"""
import numpy as np

from . import structure

SQRT2 = np.sqrt(2.0)


def butterfly_matrix(m, mu, nu):
    """O^<m>_{mu,nu} of Eq. 2 (dense, m = 2 mu + nu)."""
    assert 2 * mu + nu == m
    O = np.zeros((m, m))
    for t in range(mu):
        O[t, t] = 1.0 / SQRT2
        O[t, mu + nu + t] = 1.0 / SQRT2
        O[mu + nu + t, t] = 1.0 / SQRT2
        O[mu + nu + t, mu + nu + t] = -1.0 / SQRT2
    for t in range(nu):
        O[mu + t, mu + t] = 1.0
    return O


def layer_matrix(n, d, layer, granule=1):
    """O_layer: block-diagonal of the layer's butterflies (Eq. 3)."""
    O = np.zeros((n, n))
    covered = 0
    for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer, granule):
        size = 2 * mu + nu
        # A butterfly's rows are contiguous: [s, s + 2mu + nu), top half first,
        # the pair partner of s+t is s+h+t = s+mu+nu+t when the bottom half is
        # full, and the bottom half is truncated only in the last butterfly.
        assert s == covered
        assert mu == 0 or h == mu + nu
        O[s:s + size, s:s + size] = butterfly_matrix(size, mu, nu)
        covered += size
    assert covered == n
    return O


def dense_rbt(n, d, coeff, granule=1):
    """Dense U = O_d R_d ... O_1 R_1 (Eq. 3) from packed coefficients (n x d)."""
    Umat = np.eye(n)
    for layer in range(1, d + 1):
        Umat = layer_matrix(n, d, layer, granule) @ np.diag(coeff[:, layer - 1]) @ Umat
    return Umat


def dense_rbt_recursive_parker(coeff):
    """Parker RBT built by the recursion of Lemma 2: U = (U_0 (+) U_1) O R.

    Valid when 2^depth divides n (every butterfly is a Parker butterfly).
    coeff is the packed n x depth array of the sub-range; the children use
    the top and bottom halves of layers 2..depth.
    """
    n, depth = coeff.shape
    if depth == 0:
        return np.eye(n)
    assert n % 2 == 0
    half = n // 2
    O = np.block([[np.eye(half), np.eye(half)], [np.eye(half), -np.eye(half)]]) / SQRT2
    R = np.diag(coeff[:, 0])
    top = dense_rbt_recursive_parker(coeff[:half, 1:])
    bot = dense_rbt_recursive_parker(coeff[half:, 1:])
    Z = np.zeros((half, half))
    return np.block([[top, Z], [Z, bot]]) @ O @ R


def _pairs(n, d, layer, granule=1):
    a, b = [], []
    for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer, granule):
        a.extend(range(s, s + mu))
        b.extend(range(s + h, s + h + mu))
    return np.array(a, dtype=np.int64), np.array(b, dtype=np.int64)


def _mix_rows(X, a, b):
    xa = X[a].copy()
    xb = X[b].copy()
    X[a] = (xa + xb) / SQRT2
    X[b] = (xa - xb) / SQRT2


def apply_transpose_left(X, coeff, d, granule=1):
    """Return coeff-RBT^T @ X for X of shape (n,) or (n, k); O(d n k) work."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = X.shape[0]
    for layer in range(d, 0, -1):
        a, b = _pairs(n, d, layer, granule)
        _mix_rows(X, a, b)
        c = coeff[:, layer - 1]
        X *= c if X.ndim == 1 else c[:, None]
    return X


def apply_left(X, coeff, d, granule=1):
    """Return coeff-RBT @ X (the undo order: scale, then mix, l = 1..d)."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = X.shape[0]
    for layer in range(1, d + 1):
        c = coeff[:, layer - 1]
        X *= c if X.ndim == 1 else c[:, None]
        a, b = _pairs(n, d, layer, granule)
        _mix_rows(X, a, b)
    return X


def two_sided(A, U, V, d, granule=1):
    """A~ = U^T A V by packed butterflies (Eq. 1): rows with U, columns with V."""
    T = apply_transpose_left(A, U, d, granule)
    return apply_transpose_left(T.T, V, d, granule).T.copy()


def two_sided_dense(A, U, V, d, granule=1):
    """A~ = U^T A V with the explicit dense factors (small n only)."""
    n = A.shape[0]
    Ud = dense_rbt(n, d, U, granule)
    Vd = dense_rbt(n, d, V, granule)
    return Ud.T @ A @ Vd
