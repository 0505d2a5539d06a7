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


# ---- rotation butterflies (Sec. 3: block rotations, R_l = I) ----
#
# Layer matrix: every butterfly is [[C, 0, S], [0, I, 0], [S, 0, -C]] with
# C = diag(cos t), S = diag(sin t) over its mu pairs (rotation of 0 degrees,
# the identity, on the nu unpaired rows); U = O_d ... O_1 with no diagonal
# factors. Each O_l is symmetric and orthogonal, so U^T x applies layers
# d..1 and U x layers 1..d, each mixing a pair (a, b) into
# (c x_a + s x_b, s x_a - c x_b). Packed coefficients: coeffs.generate_rotations.


def rotation_layer_matrix(n, d, layer, coeff, granule=1):
    """Dense O_layer of the rotation RBT from packed cos/sin coefficients."""
    O = np.eye(n)
    for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer, granule):
        for t in range(mu):
            a, b = s + t, s + h + t
            c, sn = coeff[a, layer - 1], coeff[b, layer - 1]
            O[a, a], O[a, b], O[b, a], O[b, b] = c, sn, sn, -c
    return O


def dense_rotation_rbt(n, d, coeff, granule=1):
    """Dense U = O_d ... O_1 of the rotation RBT."""
    Umat = np.eye(n)
    for layer in range(1, d + 1):
        Umat = rotation_layer_matrix(n, d, layer, coeff, granule) @ Umat
    return Umat


def _rotate_rows(X, a, b, c, s):
    xa = X[a].copy()
    xb = X[b].copy()
    if X.ndim == 1:
        X[a] = c * xa + s * xb
        X[b] = s * xa - c * xb
    else:
        X[a] = c[:, None] * xa + s[:, None] * xb
        X[b] = s[:, None] * xa - c[:, None] * xb


def rotation_apply_transpose_left(X, coeff, d, granule=1):
    """coeff-rotation-RBT^T @ X (layers d..1)."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = X.shape[0]
    for layer in range(d, 0, -1):
        a, b = _pairs(n, d, layer, granule)
        _rotate_rows(X, a, b, coeff[a, layer - 1], coeff[b, layer - 1])
    return X


def rotation_apply_left(X, coeff, d, granule=1):
    """coeff-rotation-RBT @ X (layers 1..d)."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = X.shape[0]
    for layer in range(1, d + 1):
        a, b = _pairs(n, d, layer, granule)
        _rotate_rows(X, a, b, coeff[a, layer - 1], coeff[b, layer - 1])
    return X


def transform_pair(kind):
    """(U^T x, U x) routines of a butterfly kind: "diag" (Eq. 3, random
    diagonals and the butterflies of Eq. 2) or "rotation"."""
    if kind == "rotation":
        return rotation_apply_transpose_left, rotation_apply_left
    return apply_transpose_left, apply_left


def two_sided_kind(A, U, V, d, kind="diag", granule=1, sides=2):
    """A~ = U^T A V (sides = 2) or U^T A (sides = 1, the one-sided RBT of
    Sec. 7) for either butterfly kind."""
    fwd, _ = transform_pair(kind)
    T = fwd(A, U, d, granule)
    if sides == 1:
        return T
    return fwd(T.T, V, d, granule).T.copy()
