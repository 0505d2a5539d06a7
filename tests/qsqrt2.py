"""Exact arithmetic in the field Q(sqrt 2) for tiny-n checks.

Butterfly entries are 0, 1 and +-1/sqrt(2), so with rational coefficients and
a rational matrix every quantity of the method lies in Q(sqrt 2) = {a + b sqrt2}.
Test helper only (not part of the oracle or of the product).
"""
from fractions import Fraction


class Q2:
    __slots__ = ("a", "b")

    def __init__(self, a=0, b=0):
        self.a = Fraction(a)
        self.b = Fraction(b)

    @staticmethod
    def lift(x):
        return x if isinstance(x, Q2) else Q2(x, 0)

    def __add__(self, o):
        o = Q2.lift(o)
        return Q2(self.a + o.a, self.b + o.b)

    __radd__ = __add__

    def __neg__(self):
        return Q2(-self.a, -self.b)

    def __sub__(self, o):
        return self + (-Q2.lift(o))

    def __rsub__(self, o):
        return Q2.lift(o) - self

    def __mul__(self, o):
        o = Q2.lift(o)
        return Q2(self.a * o.a + 2 * self.b * o.b, self.a * o.b + self.b * o.a)

    __rmul__ = __mul__

    def inv(self):
        den = self.a * self.a - 2 * self.b * self.b
        if den == 0:
            raise ZeroDivisionError
        return Q2(self.a / den, -self.b / den)

    def __truediv__(self, o):
        return self * Q2.lift(o).inv()

    def is_zero(self):
        return self.a == 0 and self.b == 0

    def __eq__(self, o):
        o = Q2.lift(o)
        return self.a == o.a and self.b == o.b

    def __float__(self):
        return float(self.a) + float(self.b) * 2.0 ** 0.5


INV_SQRT2 = Q2(0, Fraction(1, 2))


def matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), Q2()) for j in range(m)] for i in range(n)]


def transpose(A):
    return [list(r) for r in zip(*A)]


def eye(n):
    return [[Q2(1 if i == j else 0) for j in range(n)] for i in range(n)]


def leading_pivots(A):
    """Pivots of elimination without pivoting, in exact arithmetic.
    The k-th pivot is det(A[:k,:k]) / det(A[:k-1,:k-1]); a zero pivot means a
    singular leading block.  Stops at the first zero."""
    M = [row[:] for row in A]
    n = len(M)
    piv = []
    for k in range(n):
        p = M[k][k]
        piv.append(p)
        if p.is_zero():
            break
        for i in range(k + 1, n):
            f = M[i][k] / p
            for j in range(k, n):
                M[i][j] = M[i][j] - f * M[k][j]
    return piv


def solve(A, b):
    """Exact solve with row exchanges (Gauss-Jordan on a copy)."""
    n = len(A)
    M = [A[i][:] + [b[i]] for i in range(n)]
    for k in range(n):
        p = next(i for i in range(k, n) if not M[i][k].is_zero())
        M[k], M[p] = M[p], M[k]
        for i in range(n):
            if i != k and not M[i][k].is_zero():
                f = M[i][k] / M[k][k]
                M[i] = [M[i][j] - f * M[k][j] for j in range(n + 1)]
    return [M[i][n] / M[i][i] for i in range(n)]
